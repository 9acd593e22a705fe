"""EMCCD camera on the GPU (the Discussion's electron-multiplication stage as
an extra latent: photoelectrons phi ~ Poisson(mu), register output
x ~ Gamma(phi, 1) for phi >= 1, reading w = o + G x, read noise on the
zero-photon reading) against the FP64 oracle, through the C ABI.

Per-pixel log-likelihoods on the GPU's own mu (the closed form with log I_1
against the oracle's photoelectron sum, across the power-series / asymptotic
switch of log I_1, to the FP32 rounding of the hook's output), Delta and accept decisions of colour passes, block phases
and block moves from a shared state (tie band as in the sCMOS parity tests),
the one-pixel posterior against quadrature (and Exp(1) where the reading lies
at or below the offset), posterior means of a small frame against an oracle
run, and the refusal of the scans that take
the sCMOS reading only.
"""

import math
import os
import sys

import numpy as np
import pytest

import oracle
from paper_2411_00991_amd import synth

pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from test_gpu_parity import _block_decisions, _decision_check  # noqa: E402

EM = 1                           # camera code of both sides (BDC_CAMERA_EMCCD, oracle.CAMERA_EMCCD)


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def bdc():
    import torch
    torch.cuda.set_device(0)
    import paper_2411_00991_amd as m
    assert m.BDC_CAMERA_EMCCD == EM and oracle.CAMERA_EMCCD == EM
    return m


def f32(a):
    return np.asarray(a, np.float32)


def make_problem(H, W, psf, per_pixel, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    truth = np.full((H, W), 2.0 * scale)
    synth.add_beads(truth, rng, max(1, H * W // 60), scale=50.0 * scale)
    synth.add_filaments(truth, rng, max(1, H // 24), scale=30.0 * scale)
    cam = synth.scmos_maps(rng, H, W) if per_pixel else synth.scalar_camera()
    img = synth.simulate_frame_emccd(truth, psf, cam, rng)
    g, o, s = cam.maps(H, W)
    return dict(img=f32(img), psf=f32(psf), g=f32(g), o=f32(o), s=f32(s), truth=truth, per_pixel=per_pixel)


def gpu_sampler(bdc, P, **kw):
    if P["per_pixel"]:
        cam = (P["g"], P["o"], P["s"])
    else:
        cam = (np.float32(P["g"][0, 0]), np.float32(P["o"][0, 0]), np.float32(P["s"][0, 0]))
    H, W = P["img"].shape
    return bdc.Sampler(P["psf"], *cam, height=H, width=W, camera=EM, **kw)


def oracle_sampler(P, **kw):
    d = lambda a: np.asarray(a, np.float64)
    return oracle.OracleSampler(d(P["img"]), d(P["psf"]), d(P["g"]), d(P["o"]), d(P["s"]), camera=EM, **kw)


# ---------------------------------------------------------------------------
# Log-likelihood
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", ["scalar", "per_pixel", "dim", "bright"])
def test_loglik_matches_oracle(bdc, case):
    say("EMCCD loglik", case)
    H = W = 40
    scale = {"dim": 0.02, "bright": 20.0}.get(case, 1.0)
    P = make_problem(H, W, synth.gaussian_psf(1.5, 11), case != "scalar", seed=7, scale=scale)
    S = gpu_sampler(bdc, P, n_chains=1, seed=3, schedule=bdc.BDC_SCHED_CHROMATIC)
    S.init(P["img"])
    S.sweep(2)
    ell = S.loglik(0).astype(np.float64)
    mu = S.mu()[0].astype(np.float64)            # both sides on the GPU's own mu
    want = oracle.loglik_emccd(*[P[k].astype(np.float64) for k in ("img", "g", "o", "s")], mu)
    err = np.abs(ell - want) / np.abs(want)      # the hook returns FP32: one ulp is 2^-23 relative
    c = (P["img"].astype(np.float64) - P["o"]) / P["g"]
    z = 2.0 * np.sqrt(np.maximum(c, 0.0) * mu)
    say("  max rel err %.3g; pixels at or below the offset %d; 2 sqrt(mu c) up to %.1f"
        % (err.max(), int((c <= 0).sum()), z.max()))
    assert err.max() <= 2.0 ** -23
    S.close()


def test_loglik_across_the_log_i1_switch(bdc):
    """A frame whose readings put 2 sqrt(mu c) on a fine grid through 24, where
    log I_1 changes from its power series to the asymptotic expansion, and
    out to 2000, plus readings below, at and just above the offset."""
    H, W = 16, 64
    G, o, sg = 2.0, 100.0, 1.5
    P = dict(psf=f32([[1.0]]), per_pixel=False, g=f32(np.full((H, W), G)), o=f32(np.full((H, W), o)),
             s=f32(np.full((H, W), sg)))
    z = np.concatenate([np.linspace(23.0, 25.0, 512), np.geomspace(0.01, 2000.0, 500),
                        np.zeros(12)])
    c = np.concatenate([np.full(512, 12.0), np.full(500, 6.0), [-5.0, -1e-3, 0.0, 1e-6, 1e-3, 0.02,
                                                               0.5, 1.0, 3.0, 30.0, 300.0, 3000.0]])
    mu = np.where(z > 0, z * z / (4.0 * np.maximum(c, 1e-30)), 3.7)
    w = o + G * c
    P["img"] = f32(w.reshape(H, W))
    S = gpu_sampler(bdc, P, n_chains=1, seed=1, schedule=bdc.BDC_SCHED_CHROMATIC)
    S.init(P["img"])
    rho = f32(mu.reshape(1, H, W))
    S.set_rho(rho, np.zeros_like(rho), 0)
    ell = S.loglik(0).astype(np.float64).ravel()
    mu32 = S.mu()[0].astype(np.float64).ravel()
    assert np.array_equal(mu32, rho.ravel().astype(np.float64))           # identity PSF
    want = oracle.loglik_emccd(P["img"].astype(np.float64).ravel(), G, o, sg, mu32)
    err = np.abs(ell - want) / np.abs(want)
    say("  max rel err %.3g (at z = %.4g)" % (err.max(), 2.0 * math.sqrt(max(c[err.argmax()], 0) * mu32[err.argmax()])))
    assert err.max() <= 2.0 ** -23
    S.close()


# ---------------------------------------------------------------------------
# Decisions from a shared state
# ---------------------------------------------------------------------------

CHROMATIC_CASES = {
    "gauss11_64_scalar": (64, 64, lambda: synth.gaussian_psf(1.5, 11), False, 1.0),
    "airy31_72_maps": (72, 72, lambda: synth.airy_psf(1.4, 0.6, 0.065, 31), True, 1.0),
    "gauss11_dim_maps": (48, 56, lambda: synth.gaussian_psf(1.5, 11), True, 0.05),
    "gauss11_bright_maps": (48, 56, lambda: synth.gaussian_psf(1.5, 11), True, 20.0),
    "gauss5_one_row": (1, 64, lambda: synth.gaussian_psf(1.0, 5), True, 1.0),
}


@pytest.mark.parametrize("case", list(CHROMATIC_CASES))
def test_colour_pass_decisions_match_oracle(bdc, case):
    H, W, mk, pp, scale = CHROMATIC_CASES[case]
    say("EMCCD colour pass", case)
    P = make_problem(H, W, mk(), pp, seed=11, scale=scale)
    s = P["psf"].shape[0]
    C = 2
    S = gpu_sampler(bdc, P, n_chains=C, seed=99, burn_in=3, schedule=bdc.BDC_SCHED_CHROMATIC)
    S.init(P["img"])
    S.sweep(6)
    rho, ls, t = S.rho()
    O = oracle_sampler(P, n_chains=C, seed=99, burn_in=3)
    O.init()
    errs, ties, n = [], 0, 0
    present = sorted({(y % s) * s + (x % s) for y in range(min(H, s)) for x in range(min(W, s))})
    for g in sorted(({0, 1, s + 2, (s * s) // 2, s * s - 1} | {present[0], present[-1]}) & set(present)):
        S.set_rho(rho, ls, t)
        dg, ag = S.run_groups(g, g + 1)
        O.set_state(rho.astype(np.float64), ls.astype(np.float64), t)
        do, lo, ao, sa = O.run_groups(t, g, g + 1, with_sabs=True)
        sel = ao != 255
        assert np.array_equal(sel, ag != 255)
        e, k = _decision_check(dg, ag, do, lo, ao, sa, sel)
        errs.append(e)
        ties += k
        n += int(sel.sum())
    e = np.concatenate(errs)
    say("  decisions %d, ties %d, max |dDelta|/(1+S) %.3g" % (n, ties, e.max()))
    assert n > 0 and e.max() < 1e-5
    S.close()


@pytest.mark.parametrize("B,groups,scale", [(31, (0, 961), 1.0), (31, (961 + 5, 961 + 40), 0.05),
                                            (40, (2 * 961, 2 * 961 + 200), 20.0)])
def test_block_phase_decisions_match_oracle(bdc, B, groups, scale):
    say("EMCCD block phase B=%d groups %s scale %g" % (B, groups, scale))
    P = make_problem(100, 90, synth.airy_psf(1.4, 0.6, 0.065, 31), True, seed=13, scale=scale)
    _block_decisions(bdc, P, bdc.BDC_SCHED_BLOCK, B, groups, camera=EM)


def test_block_move_decisions_match_oracle(bdc):
    """The block independence move (16 x 16 blocks, proposal around a reference
    log-density) under the EMCCD reading: Delta and decisions per block."""
    H, W, C, seed, width = 70, 52, 2, 77, 0.08
    say("EMCCD block move %dx%d" % (H, W))
    P = make_problem(H, W, synth.gaussian_psf(1.5, 11), True, seed=31)
    S = gpu_sampler(bdc, P, n_chains=C, seed=seed, burn_in=2)
    S.init(P["img"])
    S.sweep(4)
    rho, ls, t = S.rho()
    rng = np.random.default_rng(5)
    pm = f32(np.log(rho.mean(axis=0)) + 0.05 * rng.standard_normal((H, W)))
    ps = f32(np.full((H, W), width) * np.exp(0.3 * rng.standard_normal((H, W))))
    S.set_block_proposal(pm, ps)
    O = oracle_sampler(P, n_chains=C, seed=seed, burn_in=2)
    O.init()
    Pp = O.block_period()
    nbx = (W + 15) // 16
    worst, n_dec = 0.0, 0
    for k, colour in enumerate((0, 1, 3)):
        S.set_rho(rho, ls, t)
        dg, ag = S.block_colour(k + 3, colour)
        O.set_state(rho.astype(np.float64), ls.astype(np.float64), t)
        _, do, ao, sa = O.block_pass(k + 3, pm, ps, colour=colour, with_sabs=True)
        assert dg.shape == do.shape
        cy, cx = colour // Pp, colour % Pp
        nbx_c = (nbx - cx + Pp - 1) // Pp
        logu = np.empty_like(do)
        for c in range(C):
            for b in range(do.shape[1]):
                by, bx = cy + Pp * (b // nbx_c), cx + Pp * (b % nbx_c)
                logu[c, b] = math.log(oracle.uniform(seed, by * 16 * W + bx * 16, k + 3, c, 4))
        clear = np.abs(do - logu) > 1e-5 * (1.0 + sa)
        err = np.abs(dg.astype(np.float64) - do) / (1.0 + sa)
        worst = max(worst, float(err.max()))
        assert not (clear & (ag != ao)).any()
        n_dec += do.size
    say("  block decisions %d, max |dDelta|/(1+S) %.3g" % (n_dec, worst))
    assert worst < 1e-5
    S.close()


def test_moments_match_oracle_run(bdc):
    """Posterior means of a 20 x 20 EMCCD frame (Gaussian 9 x 9 PSF, scalar
    camera) under the automatic (block-phase) scan against an oracle run, per
    pixel, within the two runs' batch-means standard errors."""
    say("EMCCD moments vs oracle run (20x20, Gaussian 9x9)")
    P = make_problem(20, 20, synth.gaussian_psf(1.2, 9), False, seed=17)
    burn = 300
    O = oracle_sampler(P, n_chains=2, seed=31, burn_in=burn)
    O.init()
    O.sweep(burn)
    draws = []
    for _ in range(1200):
        O.sweep(1)
        draws.append(O.state()[0].copy())
    d = np.array(draws)                                   # [n, C, H, W]
    mo = d.mean(axis=(0, 1))
    se_o = np.sqrt(np.mean([[[oracle.batch_means_mcse(d[:, c, y, x], 30) ** 2 for x in range(20)]
                             for y in range(20)] for c in range(2)], axis=0) / 2)
    S = gpu_sampler(bdc, P, n_chains=8, seed=77, burn_in=burn, rhat_block=40, max_sweeps=3300)
    assert S.schedule_info()[1] == bdc.BDC_SCHED_BLOCK
    S.init(P["img"])
    S.sweep(3300)
    mg, _, _ = S.moments()
    se_g = S.mcse()
    z = (mg - mo) / np.sqrt(se_g ** 2 + se_o ** 2)
    frac = float((np.abs(z) > 3).mean())
    say("  frac |z|>3 = %.4f, mean z = %.3f, max |z| = %.2f" % (frac, z.mean(), np.abs(z).max()))
    assert frac <= 0.02
    assert abs(z.mean()) < 0.25
    S.close()


# ---------------------------------------------------------------------------
# One-pixel posteriors
# ---------------------------------------------------------------------------

def _posterior_by_quadrature(c, G=2.0, o=100.0, sg=1.5):
    """Mean and variance of rho = mu under a flat prior, by quadrature in
    u = log rho of the oracle's likelihood."""
    top = max(3.0 * c, c + 30.0 * math.sqrt(abs(c) + 1.0) + 50.0)
    u = np.linspace(math.log(1e-6), math.log(top), 60001)
    r = np.exp(u)
    lp = oracle.loglik_emccd(o + G * c, G, o, sg, r) + u
    p = np.exp(lp - lp.max())
    p /= p.sum()
    m = (p * r).sum()
    return m, (p * r * r).sum() - m * m


def test_one_pixel_posteriors_match_quadrature(bdc):
    """Identity PSF: every pixel is its own one-pixel problem.  Eight bands of
    512 identical pixels (readings c = (w - o)/G from below the offset to 400
    photons) give replicate chains, whose spread is the standard error of the
    band's posterior mean and variance.  At or below the offset the posterior
    is Exp(1): no photoelectron can have been amplified, so the likelihood is
    e^-mu times a constant."""
    H, W, C = 64, 64, 2
    G, o, sg = 2.0, 100.0, 1.5
    cs = [-2.0, 0.0, 0.3, 2.0, 12.0, 17.3, 60.0, 400.0]
    img = np.repeat(np.array([o + G * c for c in cs]), 8)[:, None] * np.ones((1, W))
    S = bdc.Sampler(f32([[1.0]]), np.float32(G), np.float32(o), np.float32(sg), height=H, width=W, n_chains=C,
                    seed=17, burn_in=600, camera=EM)
    S.init(f32(img))
    S.sweep(600 + 3000)
    mean, var, n = S.moments(-1)
    assert n == 3000
    for i, c in enumerate(cs):
        m_px, v_px = mean[8 * i:8 * i + 8].astype(np.float64).ravel(), var[8 * i:8 * i + 8].astype(np.float64).ravel()
        m_q, v_q = (1.0, 1.0) if c <= 0 else _posterior_by_quadrature(c, G, o, sg)
        zm = (m_px.mean() - m_q) / (m_px.std(ddof=1) / math.sqrt(m_px.size))
        zv = (v_px.mean() - v_q) / (v_px.std(ddof=1) / math.sqrt(v_px.size))
        say("  c %7.2f: mean %.5g (quadrature %.5g, z %+.2f)  var %.5g (%.5g, z %+.2f)"
            % (c, m_px.mean(), m_q, zm, v_px.mean(), v_q, zv))
        assert abs(zm) < 4.0 and abs(zv) < 4.0
    S.close()


# ---------------------------------------------------------------------------
# Scans that take the sCMOS reading only
# ---------------------------------------------------------------------------

def test_series_scans_and_their_autotune_candidates_refuse_emccd(bdc):
    psf = f32(synth.gaussian_psf(1.5, 11))
    g, o, s = np.float32(2.0), np.float32(100.0), np.float32(1.5)
    for sched in (bdc.BDC_SCHED_BLOCK_SERIES, bdc.BDC_SCHED_BLOCK9_SERIES):
        with pytest.raises(bdc.BdcError) as ei:
            bdc.Sampler(psf, g, o, s, height=64, width=64, schedule=sched, camera=EM)
        assert ei.value.status == bdc.BDC_EINVAL
    # the automatic scan: block phase, or pixel-chromatic on frames under two PSF sides
    S = bdc.Sampler(psf, g, o, s, height=64, width=64, camera=EM)
    assert S.schedule_info()[1] == bdc.BDC_SCHED_BLOCK
    small = bdc.Sampler(psf, g, o, s, height=16, width=40, camera=EM)
    assert small.schedule_info()[1] == bdc.BDC_SCHED_CHROMATIC
    small.close()
    rng = np.random.default_rng(3)
    S.init(f32(100.0 + 2.0 * rng.gamma(2.0, 5.0, (64, 64))))
    with pytest.raises(bdc.BdcError):
        S.set_schedule(bdc.BDC_SCHED_BLOCK_SERIES, 10)
    ms, best = S.autotune([-10, -11, -1005, 11, 12], 1)
    say("  autotune ms", list(ms), "best", best)
    assert all(math.isinf(m) for m in ms[:3]) and best in (11, 12)
    assert S.schedule_info()[1] == bdc.BDC_SCHED_BLOCK
    S.close()
