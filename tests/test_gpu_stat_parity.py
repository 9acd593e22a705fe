"""Statistical parity at the benchmark configurations: posterior means and
variances of the GPU's block-series sampler against an FP64 oracle run.

The oracle moments are stored under tests/golden/ (written by
make_stat_golden.py, which calls only the oracle).  Per pixel,
z = (GPU - oracle) / sqrt(se_gpu^2 + se_oracle^2) for the mean and for the
variance, standard errors from batch means over all chains on both sides.
Pass: |z| > 3 in at most 1 % of the pixels (0.27 % expected for normal z) and
the mean of z near 0.  The posterior is that of Methods, Eqs. 1-6 with the
flat separable prior.
"""

import os

import numpy as np
import pytest

from paper_2411_00991_amd import synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def bdc():
    import torch
    torch.cuda.set_device(0)
    import paper_2411_00991_amd as m
    return m


def problem(name):
    if name == "beads64":
        return synth.frame_beads_segments(64, seed=0)
    return synth.crop(synth.frame_filaments(512, seed=1), 224, 224, 64)


def _zstats(z):
    return float((np.abs(z) > 3).mean()), float(z.mean()), float(np.abs(z).max())


@pytest.mark.parametrize("name,kind", [("beads64", "series"), ("fil64", "series"), ("beads64", "series9"),
                                       ("fil64", "series9")])
def test_posterior_moments_match_oracle_run(bdc, name, kind):
    path = os.path.join(HERE, "golden", "stat_%s.npz" % name)
    if not os.path.exists(path):
        pytest.skip("oracle moments not written yet (tests/golden/make_stat_golden.py %s)" % name)
    gold = np.load(path)
    fr = problem(name)
    H, W = fr.image.shape
    s = int(fr.psf.shape[0])
    f32 = lambda a: np.asarray(a, np.float32)
    if fr.camera.per_pixel:
        cam = [f32(a) for a in fr.camera.maps(H, W)]
    else:
        cam = [np.float32(fr.camera.gain), np.float32(fr.camera.offset), np.float32(fr.camera.sigma)]
    C, burn, n, batch = 64, 300, 1600, 100
    sched, B = ((bdc.BDC_SCHED_BLOCK_SERIES, s) if kind == "series" else (bdc.BDC_SCHED_BLOCK9_SERIES, s // 2))
    say("%s: %d chains, %d + %d sweeps, %s B = %d" % (name, C, burn, n, kind, B))
    S = bdc.Sampler(f32(fr.psf), *cam, height=H, width=W, n_chains=C, seed=77, burn_in=burn,
                    schedule=sched, block_size=B, max_sweeps=burn + n)
    S.init(f32(fr.image))
    S.sweep(burn)
    nb = n // batch
    b1 = np.zeros((C, nb, H, W))
    b2 = np.zeros((C, nb, H, W))
    for i in range(nb * batch):
        S.sweep(1)
        r = S.rho()[0].astype(np.float64)
        b1[:, i // batch] += r
        b2[:, i // batch] += r * r
    b1 /= batch
    b2 /= batch
    mean, var, ns = S.moments()
    assert ns == n
    bm = b1.reshape(C * nb, H, W)
    bq = b2.reshape(C * nb, H, W)
    K = bm.shape[0]
    m_d = bm.mean(axis=0)
    # the library's pooled moments are those of the same draws
    np.testing.assert_allclose(mean, m_d, rtol=2e-5, atol=1e-5)
    v_d = (bq.mean(axis=0) - m_d ** 2) * (K * batch) / (K * batch - 1)
    np.testing.assert_allclose(var, v_d, rtol=2e-3, atol=1e-3)
    se_m = bm.std(axis=0, ddof=1) / np.sqrt(K)
    se_v = (bq - 2.0 * m_d * bm + m_d ** 2).std(axis=0, ddof=1) / np.sqrt(K)
    zm = (mean - gold["mean"]) / np.sqrt(se_m ** 2 + gold["se_mean"].astype(np.float64) ** 2)
    zv = (var - gold["var"]) / np.sqrt(se_v ** 2 + gold["se_var"].astype(np.float64) ** 2)
    fm, mm, xm = _zstats(zm)
    fv, mv, xv = _zstats(zv)
    say("  mean: frac |z|>3 %.4f, mean z %.3f, max |z| %.2f; var: frac %.4f, mean z %.3f, max |z| %.2f" % (
        fm, mm, xm, fv, mv, xv))
    say("  oracle: %d chains x %d sweeps; median se ratio (oracle/gpu) mean %.2f var %.2f" % (
        int(gold["chains"]), int(gold["sweeps"]), np.median(gold["se_mean"] / se_m), np.median(gold["se_var"] / se_v)))
    assert fm <= 0.01 and abs(mm) < 0.2
    assert fv <= 0.01 and abs(mv) < 0.2
    S.close()
