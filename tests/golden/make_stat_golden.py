"""Writes the oracle's posterior moments for the statistical parity tests.

Calls only the FP64 oracle (``oracle/``) and the seeded input generators.
Each case runs independent oracle chains (one process each, one thread, a
distinct Philox seed per chain), discards the burn-in (step adaptation), then
records every sweep's rho in batches of `batch` sweeps.  Per pixel it stores
the pooled posterior mean and variance (Methods, Prior: the posterior of
Eq. 9 with the flat separable prior) and their Monte Carlo standard errors
from the batch means over all chains:

  mean    = average of all draws;       se_mean = sd(batch means of rho) / sqrt(#batches)
  var     = unbiased sample variance;   se_var  = sd(batch means of (rho - mean)^2) / sqrt(#batches)

Cases:
  beads64   the 64 x 64 frame (Gaussian PSF sigma 1.5 px, 11 x 11, 20 beads and
            segments on 2 photons/px, scalar camera G 2, o 100, sigma 1.5), seed 0;
  fil64     the central 64 x 64 window of the 512 x 512 filament frame (Airy
            31 x 31, per-pixel sCMOS maps), seed 1.

Both chains use the block-phase scan with B = PSF side (the block-series
scan visits pixels in the same order).

    python tests/golden/make_stat_golden.py beads64 [--procs 6]
"""

from __future__ import annotations

import argparse
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

CASES = {
    # name: (chains, burn_in, sampled sweeps, batch, base seed)
    "beads64": (12, 300, 1500, 100, 1000),
    "fil64": (8, 400, 2000, 100, 2000),
}


def problem(name):
    from paper_2411_00991_amd import synth
    if name == "beads64":
        return synth.frame_beads_segments(64, seed=0)
    if name == "fil64":
        return synth.crop(synth.frame_filaments(512, seed=1), 224, 224, 64)
    raise KeyError(name)


def run_chain(args):
    name, k = args
    import oracle
    oracle.set_threads(1)
    C, burn, n, batch, base = CASES[name]
    fr = problem(name)
    H, W = fr.image.shape
    g, o, s = fr.camera.maps(H, W)
    f64 = lambda a: np.asarray(np.asarray(a, np.float32), np.float64)   # the inputs the GPU sees
    S = oracle.OracleSampler(f64(fr.image), f64(fr.psf), f64(g), f64(o), f64(s), n_chains=1, seed=base + k,
                             burn_in=burn, schedule=oracle.SCHED_BLOCK, block=int(fr.psf.shape[0]))
    S.init()
    t0 = time.time()
    S.sweep(burn)
    nb = n // batch
    b1 = np.zeros((nb, H, W))
    b2 = np.zeros((nb, H, W))
    for i in range(nb * batch):
        S.sweep(1)
        r = S.state()[0][0]
        b1[i // batch] += r
        b2[i // batch] += r * r
    print("  %s chain %d done in %.0f s" % (name, k, time.time() - t0), flush=True)
    return b1 / batch, b2 / batch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("case", choices=sorted(CASES))
    ap.add_argument("--procs", type=int, default=6)
    a = ap.parse_args()
    C, burn, n, batch, base = CASES[a.case]
    with mp.get_context("spawn").Pool(a.procs) as pool:
        res = pool.map(run_chain, [(a.case, k) for k in range(C)])
    bm = np.concatenate([r[0] for r in res])          # [C * nb, H, W] batch means of rho
    bq = np.concatenate([r[1] for r in res])          # ... of rho^2
    K = bm.shape[0]
    ndraw = K * batch
    mean = bm.mean(axis=0)
    var = (bq.mean(axis=0) - mean ** 2) * ndraw / (ndraw - 1)
    se_mean = bm.std(axis=0, ddof=1) / np.sqrt(K)
    y = bq - 2.0 * mean * bm + mean ** 2              # batch means of (rho - mean)^2
    se_var = y.std(axis=0, ddof=1) / np.sqrt(K)
    out = os.path.join(HERE, "stat_%s.npz" % a.case)
    np.savez_compressed(out, mean=mean.astype(np.float32), var=var.astype(np.float32),
                        se_mean=se_mean.astype(np.float32), se_var=se_var.astype(np.float32),
                        chains=C, burn_in=burn, sweeps=n, batch=batch, base_seed=base)
    print("wrote", out, "batches", K)


if __name__ == "__main__":
    main()
