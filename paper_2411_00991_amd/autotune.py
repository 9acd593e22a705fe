"""Scan autotuner with a persistent cache.

The timing itself is bdc_autotune (real sweeps timed with HIP events in the
library); this module picks the candidates, groups problems into classes and
keeps the winners in a JSON file keyed by device name, so later runs apply a
cached choice with bdc_set_schedule instead of re-timing.

A class is (PSF side, frame side rounded up to a power of two, chains,
which scans are allowed).  Candidates are encoded as in bdc_autotune: 0 the
pixel-chromatic scan, B > 0 the block-phase scan with block side B, -B the
block-series scan with block side B, -(1000 + B) the nine-phase block-series
scan with block side B.  The cache lives at $BDC_AUTOTUNE_CACHE, else
~/.cache/bdc/autotune.json.
"""

from __future__ import annotations

import json
import os
from typing import Dict, Iterable, List, Optional

from . import (BDC_CAMERA_SCMOS, BDC_SCHED_BLOCK, BDC_SCHED_BLOCK9_SERIES, BDC_SCHED_BLOCK_SERIES,
               BDC_SCHED_CHROMATIC, Sampler)

NINE = 1000                     # candidate -(NINE + B): the nine-phase block-series scan


def cache_path() -> str:
    p = os.environ.get("BDC_AUTOTUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "bdc", "autotune.json")


def device_name() -> str:
    try:
        import torch
        return torch.cuda.get_device_name(0)
    except Exception:
        return "unknown-device"


def _pow2(n: int) -> int:
    return 1 << max(0, (int(n) - 1).bit_length())


def problem_class(s: int, height: int, width: int, chains: int, allow_chromatic: bool,
                  allow_series: bool = True, allow_nine: bool = True) -> str:
    kind = (("chromatic+" if allow_chromatic else "") + ("series+" if allow_series else "")
            + ("nine+" if allow_series and allow_nine else "") + "block")
    return "s%d_side%d_c%d_%s" % (s, _pow2(max(height, width)), chains, kind)


def candidates(s: int, allow_chromatic: bool = True, allow_series: bool = True,
               allow_nine: bool = True) -> List[int]:
    """Block-phase sides from psf side - 1 to 2 psf sides, the block-series scan
    at sides psf side - 1 and psf side (negative), the nine-phase block-series
    scan at sides (psf side - 1)/2 rounded up and psf side, and 0 = chromatic."""
    c = sorted({max(1, s - 1), s, s + 1, (3 * s) // 2, 2 * s})
    ser = [-b for b in sorted({max(1, s - 1), s})] if allow_series and s <= 31 else []
    nine = ([-(NINE + b) for b in sorted({max(1, s // 2), s})]
            if allow_series and allow_nine and s <= 31 else [])
    return ([0] if allow_chromatic else []) + ser + nine + c


def decode(b: int):
    """(schedule, block side) of candidate code b."""
    if b == 0:
        return BDC_SCHED_CHROMATIC, 0
    if b <= -NINE:
        return BDC_SCHED_BLOCK9_SERIES, -b - NINE
    if b < 0:
        return BDC_SCHED_BLOCK_SERIES, -b
    return BDC_SCHED_BLOCK, b


def apply(sampler: Sampler, b: int) -> None:
    """Set the scan that candidate code b stands for."""
    sampler.set_schedule(*decode(b))


def load_cache(path: Optional[str] = None) -> Dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(data: Dict, path: Optional[str] = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(sampler: Sampler, s: int, allow_chromatic: bool = True, sweeps: int = 2,
         use_cache: bool = True, path: Optional[str] = None, allow_series: bool = True,
         allow_nine: bool = True) -> int:
    """Best scan for this sampler's class (candidate code, see the module doc),
    applied to it.  Timing runs real sweeps (they advance the chain), so call
    it during burn-in.  An EMCCD sampler has no block-series candidates."""
    if sampler.cfg.camera != BDC_CAMERA_SCMOS:
        allow_series = False
    key = problem_class(s, sampler.H, sampler.W, sampler.C, allow_chromatic, allow_series, allow_nine)
    dev = device_name()
    cache = load_cache(path) if use_cache else {}
    hit = cache.get(dev, {}).get(key)
    if hit is not None:
        b = int(hit["block"])
        apply(sampler, b)
        return b
    cands = candidates(s, allow_chromatic, allow_series, allow_nine)
    ms, best = sampler.autotune(cands, sweeps)
    if best == -(2 ** 31):
        return best
    if use_cache:
        cache.setdefault(dev, {})[key] = {"block": int(best),
                                          "ms_per_sweep": {str(c): float(m) for c, m in zip(cands, ms)}}
        save_cache(cache, path)
    return best


def tune_tiles(samplers: Iterable[Sampler], psf_sides: Iterable[int], sweeps: int = 1,
               use_cache: bool = True, path: Optional[str] = None) -> Dict[str, int]:
    """Tune one representative tile per class (block-phase and block-series
    scans: the batch runs no chromatic scan) and apply the winner to every tile
    of the class."""
    groups: Dict[str, List] = {}
    for sp, s in zip(samplers, psf_sides):
        groups.setdefault(problem_class(s, sp.H, sp.W, sp.C, False, True, True), []).append((sp, s))
    chosen = {}
    for key, members in groups.items():
        rep, s = members[0]
        b = tune(rep, s, allow_chromatic=False, sweeps=sweeps, use_cache=use_cache, path=path)
        for sp, _ in members[1:]:
            apply(sp, b)
        chosen[key] = b
    return chosen
