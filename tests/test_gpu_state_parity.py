"""GPU (HIP) against the FP64 oracle for the parts of a sweep that decision
parity at t >= burn_in does not reach: the default initial state, the
per-pixel step adaptation during burn-in, the Gamma prior (Methods, Prior:
the posterior of Eq. 9 with a separable prior), and the training pairs the
learned part derives from the posterior moments.
"""

import os
import sys

import numpy as np
import pytest

import oracle
from paper_2411_00991_amd import synth

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from test_gpu_parity import make_problem, gpu_sampler, oracle_sampler, f32  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def bdc():
    import torch
    torch.cuda.set_device(0)
    import paper_2411_00991_amd as m
    return m


@pytest.mark.parametrize("per_pixel", [False, True])
def test_default_initial_state_matches_oracle(bdc, per_pixel):
    """rho0_m = max(c_m, 1/2) exp(xi_m / 2), xi from stream 2 at sweep 0 per
    chain, and every log step = log_step0 (element by element)."""
    say("default rho0, per-pixel camera" if per_pixel else "default rho0, scalar camera")
    P = make_problem(37, 45, synth.gaussian_psf(1.5, 11), per_pixel, seed=61)
    C = 3
    S = gpu_sampler(bdc, P, n_chains=C, seed=0x1234_5678_9ABC, log_step0=-1.25)
    S.init(P["img"])
    rho, ls, t = S.rho()
    O = oracle_sampler(P, n_chains=C, seed=0x1234_5678_9ABC, log_step0=-1.25)
    O.init()
    ro, lo_, _, to = O.state()
    assert t == to == 0
    err = np.abs(rho - ro) / ro
    say("  max rel err %.3g" % err.max())
    # FP32 Box-Muller and exp: a few ulp of xi, times |xi|/2 <= 3
    assert err.max() < 5e-6
    assert np.all(ls == np.float32(-1.25)) and np.all(lo_ == -1.25)
    S.close()


def _run_and_compare(bdc, P, *, schedule, B, groups, burn_in, sweeps, seed, C=2, prior=None):
    """One range of schedule groups from a shared state at sweep `sweeps`:
    decisions equal outside the tie band (and, inside a block, up to its first
    tie), committed rho and log steps element by element."""
    H, W = P["img"].shape
    s = P["psf"].shape[0]
    pk = {} if prior is None else dict(prior_kind=bdc.BDC_PRIOR_GAMMA, prior_a=prior[0], prior_b=prior[1])
    po = {} if prior is None else dict(prior_kind=oracle.PRIOR_GAMMA, prior_a=prior[0], prior_b=prior[1])
    S = gpu_sampler(bdc, P, n_chains=C, seed=seed, burn_in=burn_in, schedule=schedule, block_size=B, **pk)
    sched_o = oracle.SCHED_CHROMATIC if schedule == bdc.BDC_SCHED_CHROMATIC else oracle.SCHED_BLOCK
    O = oracle_sampler(P, n_chains=C, seed=seed, burn_in=burn_in, schedule=sched_o, block=B, **po)
    S.init(P["img"])
    S.sweep(sweeps)
    rho, ls, t = S.rho()
    assert t == sweeps
    O.init()
    g0, g1 = groups
    S.set_rho(rho, ls, t)
    dg, ag = S.run_groups(g0, g1)
    O.set_state(rho.astype(np.float64), ls.astype(np.float64), t)
    do, lu, ao, sa = O.run_groups(t, g0, g1, with_sabs=True)
    sel = ao != 255
    assert np.array_equal(sel, ag != 255)
    tie = sel & (np.abs(do - lu) <= 1e-5 * (1.0 + sa))
    keep = sel.copy()
    if tie.any():
        if schedule == bdc.BDC_SCHED_CHROMATIC:
            keep &= ~tie
        else:
            for c, y, x in zip(*np.nonzero(tie)):
                by, bx = y // B, x // B
                g_tie = ((y - by * B) % s) * s + ((x - bx * B) % s)
                yy, xx = np.mgrid[by * B:min((by + 1) * B, H), bx * B:min((bx + 1) * B, W)]
                later = ((yy - by * B) % s) * s + ((xx - bx * B) % s) >= g_tie
                keep[c, yy[later], xx[later]] = False
    assert np.array_equal(ag[keep], ao[keep]), "decision mismatch outside the tie band"
    err = np.abs(dg[keep].astype(np.float64) - do[keep]) / (1.0 + sa[keep])
    assert err.max() < 1e-5
    rg, lg, _ = S.rho()
    ro, lso, _, _ = O.state()
    np.testing.assert_allclose(rg[keep], ro[keep], rtol=2e-6)
    # log steps: every pixel of the range moved by (t+1)^-0.6 (1[acc] - 0.44)
    # during burn-in, the others kept theirs
    np.testing.assert_allclose(lg[keep], lso[keep], rtol=1e-6, atol=1e-6)
    np.testing.assert_array_equal(lg[~sel], ls[~sel])
    moved = np.abs(lg[keep] - ls[keep])
    if sweeps < burn_in:
        gain = (sweeps + 1.0) ** -0.6
        np.testing.assert_allclose(moved, np.where(ao[keep] == 1, 0.56, 0.44) * gain, rtol=1e-5)
    else:
        assert np.all(moved == 0)
    say("  decisions %d (ties %d), accepted %d, max |dDelta|/(1+S) %.3g" % (
        keep.sum(), tie.sum(), int(ao[keep].sum()), err.max()))
    S.close()


ADAPT_CASES = {
    # name: (H, W, psf, per-pixel maps, schedule, B, groups)
    "chromatic_gauss11": (64, 64, lambda: synth.gaussian_psf(1.5, 11), False, "chromatic", 0, (17, 18)),
    "block_airy31": (80, 70, lambda: synth.airy_psf(1.4, 0.6, 0.065, 31), True, "block", 31, (961, 961 + 120)),
    "series_airy31": (80, 70, lambda: synth.airy_psf(1.4, 0.6, 0.065, 31), True, "series", 31, (0, 961)),
    "series_gauss11": (64, 64, lambda: synth.gaussian_psf(1.5, 11), False, "series", 11, (121, 2 * 121)),
}


@pytest.mark.parametrize("case", list(ADAPT_CASES))
def test_step_adaptation_during_burn_in_matches_oracle(bdc, case):
    H, W, mk, pp, sched, B, groups = ADAPT_CASES[case]
    say("step adaptation at t < burn_in:", case)
    P = make_problem(H, W, mk(), pp, seed=71)
    schedule = {"chromatic": bdc.BDC_SCHED_CHROMATIC, "block": bdc.BDC_SCHED_BLOCK,
                "series": bdc.BDC_SCHED_BLOCK_SERIES}[sched]
    _run_and_compare(bdc, P, schedule=schedule, B=B, groups=groups, burn_in=50, sweeps=4, seed=19)


def test_step_is_frozen_after_burn_in(bdc):
    say("log steps frozen at t >= burn_in (block-series)")
    P = make_problem(64, 64, synth.gaussian_psf(1.5, 11), False, seed=72)
    _run_and_compare(bdc, P, schedule=bdc.BDC_SCHED_BLOCK_SERIES, B=11, groups=(0, 121), burn_in=3,
                     sweeps=5, seed=21)


@pytest.mark.parametrize("sched", ["chromatic", "series"])
def test_gamma_prior_decisions_match_oracle(bdc, sched):
    """Prior and Hastings terms with a Gamma(a, b) prior: (a - 1) log(rho'/rho)
    - b (rho' - rho) enters Delta on both sides."""
    say("Gamma prior decisions:", sched)
    P = make_problem(64, 64, synth.gaussian_psf(1.5, 11), True, seed=73)
    schedule = bdc.BDC_SCHED_CHROMATIC if sched == "chromatic" else bdc.BDC_SCHED_BLOCK_SERIES
    groups = (40, 41) if sched == "chromatic" else (0, 121)
    _run_and_compare(bdc, P, schedule=schedule, B=0 if sched == "chromatic" else 11, groups=groups,
                     burn_in=2, sweeps=3, seed=23, prior=(2.5, 0.04))


def test_gamma_prior_identity_psf_matches_closed_form(bdc):
    """Identity PSF: every pixel is a 1-pixel problem whose posterior under a
    Gamma(a, b) prior is a mixture of Gamma(a + phi, b + 1) (closed form)."""
    from test_oracle_pins import one_pixel_posterior
    say("Gamma prior, identity PSF closed form")
    rng = np.random.default_rng(31)
    H = W = 16
    truth = rng.gamma(2.0, 15.0, (H, W)) + 1.0
    cam = synth.scmos_maps(rng, H, W)
    psf = np.array([[1.0]])
    img = f32(synth.simulate_frame(truth, psf, cam, rng))
    g, o, s = [f32(a) for a in cam.maps(H, W)]
    a, b = 3.0, 0.08
    exact = np.array([[one_pixel_posterior(float(img[y, x]), float(g[y, x]), float(o[y, x]), float(s[y, x]), a, b)
                       for x in range(W)] for y in range(H)])
    S = bdc.Sampler(f32(psf), g, o, s, height=H, width=W, n_chains=8, seed=4, burn_in=500,
                    prior_kind=bdc.BDC_PRIOR_GAMMA, prior_a=a, prior_b=b, rhat_block=50, max_sweeps=4500)
    S.init(img)
    S.sweep(4500)
    mean, var, n = S.moments()
    se = S.mcse()
    z = (mean - exact[..., 0]) / se
    say("  n=%d max|z|=%.2f mean z=%.3f" % (n, np.abs(z).max(), z.mean()))
    assert np.all(np.abs(z) < 4.5)
    assert abs(z.mean()) < 0.3
    np.testing.assert_allclose(var, exact[..., 1], rtol=0.15)
    S.close()


def test_training_targets_match_their_definition(bdc):
    """x = c / scale and target = (log m - s2/2 - log scale, log(s2)/2) with
    s2 = log(1 + v/m^2), (m, v) the pooled posterior moments the library
    reports and scale = mean c (c = (w - o)/G), in double precision here."""
    say("training targets")
    P = make_problem(48, 40, synth.gaussian_psf(1.5, 11), True, seed=74)
    S = gpu_sampler(bdc, P, n_chains=2, seed=5, burn_in=20)
    S.init(P["img"])
    S.sweep(60)
    m, v, n = S.moments()
    assert n == 40
    x, tgt, sc = S.training_targets()
    c = (P["img"].astype(np.float64) - P["o"]) / P["g"]
    want_sc = c.mean()
    assert sc == pytest.approx(want_sc, rel=1e-5)
    np.testing.assert_allclose(x, c / want_sc, rtol=2e-6, atol=1e-6)
    m = m.astype(np.float64)
    v = v.astype(np.float64)
    s2 = np.log1p(v / m ** 2)
    np.testing.assert_allclose(tgt[..., 0], np.log(m) - 0.5 * s2 - np.log(want_sc), rtol=0, atol=2e-5)
    np.testing.assert_allclose(tgt[..., 1], 0.5 * np.log(s2), rtol=0, atol=2e-5)
    S.close()
