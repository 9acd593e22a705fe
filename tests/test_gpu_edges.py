"""Degenerate and extreme inputs on the GPU: a one-pixel frame under a PSF
wider than the frame (its posterior in closed form), and the largest frame
the boundary accepts (2^27 pixels), whose decisions for one colour group are
compared with the FP64 oracle's from the same state."""

import os
import sys

import numpy as np
import pytest

import oracle
from paper_2411_00991_amd import synth

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from test_gpu_parity import _decision_check  # noqa: E402

pytestmark = pytest.mark.gpu


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


def test_one_pixel_frame_under_a_wider_psf_matches_its_closed_form(bdc):
    """A 1 x 1 frame under a 5 x 5 PSF sees only the PSF's centre weight p
    (zero padding): mu = p rho, so with the flat prior the posterior of rho is
    the identity-PSF posterior of p rho scaled by 1/p (Methods, Eqs. 1-6)."""
    from test_oracle_pins import one_pixel_posterior
    psf = synth.gaussian_psf(1.0, 5)
    p = float(psf[2, 2] / psf.sum())
    G, o, sg, w = 2.0, 100.0, 1.5, 131.0
    m1, v1 = one_pixel_posterior(w, G, o, sg)
    mean, var = m1 / p, v1 / p ** 2
    S = bdc.Sampler(f32(psf), np.float32(G), np.float32(o), np.float32(sg), height=1, width=1, n_chains=8, seed=6,
                    burn_in=500, rhat_block=50, max_sweeps=6000)
    assert S.schedule_info()[1] == bdc.BDC_SCHED_CHROMATIC
    S.init(f32([[w]]))
    S.sweep(6000)
    mg, vg, n = S.moments()
    se = S.mcse()
    z = (mg[0, 0] - mean) / se[0, 0]
    say("  p = %.4f, exact mean %.3f var %.3f; gpu %.3f %.3f (n %d), z %.2f" % (p, mean, var, mg[0, 0], vg[0, 0], n,
                                                                            z))
    assert abs(z) < 4.5
    assert vg[0, 0] == pytest.approx(var, rel=0.1)
    S.close()


def test_largest_frame_one_group_matches_oracle(bdc):
    """16384 x 8192 = 2^27 pixels (the boundary's maximum frame), one chain,
    Gaussian 5 x 5 PSF, scalar camera, under the automatic scan: after two
    sweeps, one colour group's decisions and Deltas against the oracle's from
    the same state."""
    H, W = 16384, 8192
    rng = np.random.default_rng(12)
    G, o, sg = 2.0, 100.0, 1.5
    say("largest frame: building %d x %d inputs" % (H, W))
    img = (o + G * rng.poisson(6.0, (H, W)) + sg * rng.standard_normal((H, W), dtype=np.float32)).astype(np.float32)
    psf = f32(synth.gaussian_psf(1.0, 5))
    S = bdc.Sampler(psf, np.float32(G), np.float32(o), np.float32(sg), height=H, width=W, n_chains=1, seed=5,
                    burn_in=10, max_sweeps=8)
    _, sched, B = S.schedule_info()
    say("  scan %d, block %d; init + 2 sweeps" % (sched, B))
    S.init(img)
    S.sweep(2)
    rho, ls, t = S.rho()
    assert np.all(rho > 0) and np.all(np.isfinite(rho))
    say("  group 0 on the GPU")
    dg, ag = S.run_groups(0, 1)
    S.close()
    say("  group 0 on the oracle")
    osched = {bdc.BDC_SCHED_BLOCK9_SERIES: oracle.SCHED_BLOCK9, bdc.BDC_SCHED_BLOCK_SERIES: oracle.SCHED_BLOCK,
              bdc.BDC_SCHED_BLOCK: oracle.SCHED_BLOCK, bdc.BDC_SCHED_CHROMATIC: oracle.SCHED_CHROMATIC}[sched]
    O = oracle.OracleSampler(img.astype(np.float64), psf.astype(np.float64), G, o, sg, n_chains=1, seed=5,
                             burn_in=10, schedule=osched, block=B)
    O.init()
    O.set_state(rho.astype(np.float64), ls.astype(np.float64), t)
    del rho, ls
    do, lo, ao, sa = O.run_groups(t, 0, 1, with_sabs=True)
    sel = ao != 255
    assert sel.sum() > 100000 and np.array_equal(sel, ag != 255)
    err, ties = _decision_check(dg, ag, do, lo, ao, sa, sel)
    say("  %d decisions, %d ties, max |dDelta|/(1+S) %.3g" % (sel.sum(), ties, err.max()))
    assert err.max() < 1e-5
