"""Batched persistent sweeps and the autotuner, through the C ABI.

The batch must reproduce, bit for bit, what each tile's own context computes
with bdc_sweep (same kernels' arithmetic, same Philox streams), with either
camera; many tiny
tiles pooled reproduce the exact 2-pixel posterior."""

import os
import sys

import numpy as np
import pytest

from paper_2411_00991_amd import synth

pytestmark = pytest.mark.gpu
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def bdc():
    import torch
    torch.cuda.set_device(0)
    import paper_2411_00991_amd as m
    return m


def f32(a):
    return np.asarray(a, np.float32)


def tile_specs(emccd=()):
    """Six tiles of assorted shapes, PSFs and chain counts; the tiles whose
    index is in emccd read an EMCCD frame (electron-multiplying register),
    the others an sCMOS frame."""
    rng = np.random.default_rng(5)
    specs = []
    for i, (H, W, kind, s, C) in enumerate([(40, 52, "g", 9, 1), (64, 64, "a", 15, 2), (77, 45, "g", 21, 1),
                                            (96, 100, "a", 31, 2), (33, 70, "g", 11, 3), (128, 64, "a", 25, 1)]):
        psf = synth.gaussian_psf(1.0 + 0.1 * s, s) if kind == "g" else synth.airy_psf_matched(s / 10.0, s)
        truth = np.full((H, W), 3.0)
        synth.add_beads(truth, rng, H * W // 80, scale=40.0)
        cam = synth.scmos_maps(rng, H, W)
        em = i in emccd
        img = (synth.simulate_frame_emccd if em else synth.simulate_frame)(truth, psf, cam, rng)
        specs.append(dict(img=f32(img), psf=f32(psf), cam=[f32(a) for a in cam.maps(H, W)], H=H, W=W, C=C,
                          seed=1000 + i, burn_in=2 + i % 3, camera=1 if em else 0))
    return specs


def make(bdc, sp, schedule=None, **kw):
    S = bdc.Sampler(sp["psf"], *sp["cam"], height=sp["H"], width=sp["W"], n_chains=sp["C"], seed=sp["seed"],
                    burn_in=sp["burn_in"], schedule=bdc.BDC_SCHED_BLOCK if schedule is None else schedule,
                    rhat_block=2, max_sweeps=16, camera=sp.get("camera", 0), **kw)
    S.init(sp["img"])
    return S


@pytest.mark.parametrize("scan", ["block", "series", "series9", "mixed", "emccd"])
def test_batch_reproduces_separate_runs_bitwise(bdc, scan):
    # "emccd": tiles 0, 3 and 4 read EMCCD frames (block-phase scan, the only
    # batched scan that camera takes) beside sCMOS tiles of both series scans
    em = (0, 3, 4) if scan == "emccd" else ()
    specs = tile_specs(em)
    say("batch of %d tiles, %s scan" % (len(specs), scan))
    kinds = [bdc.BDC_SCHED_BLOCK, bdc.BDC_SCHED_BLOCK_SERIES, bdc.BDC_SCHED_BLOCK9_SERIES]
    if scan == "emccd":
        scheds = [kinds[0] if i in em else kinds[1 + i % 2] for i in range(len(specs))]
    else:
        scheds = [{"block": kinds[0], "series": kinds[1], "series9": kinds[2]}[scan] if scan != "mixed"
                  else kinds[i % 3] for i in range(len(specs))]
    tiles = [make(bdc, sp, sc) for sp, sc in zip(specs, scheds)]
    batch = bdc.Batch(tiles)
    n_items, grid, lds = batch.info()
    say("  items/sweep %d, grid %d, lds %d" % (n_items, grid, lds))
    batch.sweep(1)
    batch.check()
    say("  first batched sweep done")
    batch.sweep(3)
    batch.sweep(3)
    batch.check()
    say("  7 batched sweeps done")
    for i, sp in enumerate(specs):
        ref = make(bdc, sp, scheds[i])
        assert ref.schedule_info()[1] == scheds[i]
        ref.sweep(7)
        ra, la, ta = tiles[i].rho()
        rb, lb, tb = ref.rho()
        assert ta == tb == 7
        assert np.array_equal(ra, rb) and np.array_equal(la, lb), "tile %d state differs" % i
        ma, va, _ = tiles[i].moments()
        mb, vb, _ = ref.moments()
        assert np.array_equal(ma, mb) and np.array_equal(va, vb)
        assert np.array_equal(tiles[i].trace(), ref.trace())
        assert np.array_equal(tiles[i].accept_stats()[0], ref.accept_stats()[0])
        ref.close()
    # tiles stay usable on their own after batching
    tiles[0].sweep(1)
    assert tiles[0].rho()[2] == 8
    batch.close()
    for t in tiles:
        t.close()


def test_many_tiny_tiles_reproduce_two_pixel_posterior(bdc):
    from test_oracle_pins import two_pixel_posterior
    say("256 two-pixel tiles")
    w = np.array([140.0, 118.0])
    mean, var = two_pixel_posterior(w, 2.0, 100.0, 1.5)
    psf = np.zeros((3, 3), np.float32)
    psf[1] = [0.25, 0.5, 0.25]
    tiles = []
    for i in range(256):
        S = bdc.Sampler(psf, np.float32(2.0), np.float32(100.0), np.float32(1.5), height=1, width=2, n_chains=4,
                        seed=77 + i, burn_in=300, schedule=bdc.BDC_SCHED_BLOCK, block_size=2, max_sweeps=2)
        S.init(f32(w[None, :]))
        tiles.append(S)
    batch = bdc.Batch(tiles)
    batch.sweep(1300)
    batch.check()
    ms = np.array([t.moments()[0][0] for t in tiles])     # [256, 2] per-tile pooled means (4 chains x 1000)
    vs = np.array([t.moments()[1][0] for t in tiles])
    m = ms.mean(axis=0)
    se = ms.std(axis=0, ddof=1) / np.sqrt(len(tiles))
    z = (m - mean) / se
    say("  means", m, mean, "z", z)
    assert np.all(np.abs(z) < 4.0)
    np.testing.assert_allclose(vs.mean(axis=0), var, rtol=0.05)
    batch.close()
    for t in tiles:
        t.close()


def test_autotune_picks_a_valid_scan_and_keeps_sampling(bdc):
    say("autotune")
    fr = synth.frame_filaments(128, seed=4, n_filaments=10)
    g, o, s = [f32(a) for a in fr.camera.maps(128, 128)]
    S = bdc.Sampler(f32(fr.psf), g, o, s, height=128, width=128, n_chains=2, seed=3, burn_in=50)
    S.init(f32(fr.image))
    from paper_2411_00991_amd import autotune
    cands = [0, -31, -30, -1015, -1031, 30, 31, 40, 62, 200, -40, -1014]
    ms, best = S.autotune(cands, sweeps=2)
    say("  ms/sweep", dict(zip(cands, ms.tolist())), "best", best)
    # 200 > 4 * psf side; -40: series needs B <= psf side; -1014: nine phases need B >= (psf side - 1) / 2
    assert np.all(np.isinf(ms[-3:]))
    assert best in cands[:-3] and np.isfinite(ms[cands.index(best)])
    assert ms[cands.index(best)] == np.min(ms)
    n_groups, sched, B = S.schedule_info()
    assert (sched, B if best else 0) == autotune.decode(best)
    t0 = S.rho()[2]
    S.sweep(3)
    rho, _, t = S.rho()
    assert t == t0 + 3 and np.all(rho > 0)
    S.close()


def test_autotune_cache_applies_without_retiming(bdc, tmp_path, monkeypatch):
    from paper_2411_00991_amd import autotune
    monkeypatch.setenv("BDC_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    say("autotune cache")
    fr = synth.frame_beads_segments(64, seed=9)
    S = bdc.Sampler(f32(fr.psf), np.float32(2.0), np.float32(100.0), np.float32(1.5), height=64, width=64,
                    n_chains=1, seed=1, burn_in=100)
    S.init(f32(fr.image))
    b1 = autotune.tune(S, 11)
    t1 = S.rho()[2]
    assert t1 > 0                                  # timed sweeps advanced the chain
    cache = autotune.load_cache()
    assert any(b1 == v["block"] for v in cache[autotune.device_name()].values())
    S2 = bdc.Sampler(f32(fr.psf), np.float32(2.0), np.float32(100.0), np.float32(1.5), height=64, width=64,
                     n_chains=1, seed=1, burn_in=100)
    S2.init(f32(fr.image))
    b2 = autotune.tune(S2, 11)
    assert b2 == b1 and S2.rho()[2] == 0          # applied from the cache, no sweeps run
    _, sched, B = S2.schedule_info()
    assert (sched, B if b1 else 0) == autotune.decode(b1)
    S.close()
    S2.close()
