"""Object lattice finer than the pixel lattice on the GPU (Methods, Image
Formation Model, Eqs. 1-2, with k x k object cells per camera pixel and the
PSF sampled on the object lattice) against the FP64 oracle, through the C ABI.

The forward model (per-phase pixel-footprint tables folded from the object
PSF) against the oracle's convolution plus pixel integration; the default
start element by element; Delta and accept decisions of colour passes from a
shared state, single colours and runs of colours that commit pixel means
(sCMOS and EMCCD readings, ragged frames, k = 2 and 3); the one-pixel
posterior of k^2 cells against its closed form over replicate pixels;
posterior means against an oracle run (Gamma prior with sCMOS, flat prior
with EMCCD); and the refusal of what takes the pixel lattice only.
"""

import math

import numpy as np
import pytest

import oracle
from paper_2411_00991_amd import synth

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


def _pool(a, k):
    H, W = a.shape[-2] // k, a.shape[-1] // k
    return a.reshape(a.shape[:-2] + (H, k, W, k)).sum(axis=(-3, -1))


def make_problem(H, W, k, psf, per_pixel, seed, emccd=False, scale=1.0):
    """A k-times finer synthetic object (beads and filaments at the object
    lattice's scale) imaged onto an H x W camera."""
    from scipy import signal
    rng = np.random.default_rng(seed)
    truth = np.full((k * H, k * W), 2.0 * scale / (k * k))
    synth.add_beads(truth, rng, max(1, H * W // 40), scale=40.0 * scale / (k * k))
    synth.add_filaments(truth, rng, max(1, H // 12), scale=20.0 * scale / (k * k))
    mu = np.clip(_pool(signal.convolve2d(truth, psf / psf.sum(), mode="same"), k), 0.0, None)
    cam = synth.scmos_maps(rng, H, W) if per_pixel else synth.scalar_camera()
    g, o, sg = cam.maps(H, W)
    phi = rng.poisson(mu)
    if emccd:
        x = np.where(phi > 0, rng.gamma(np.maximum(phi, 1), 1.0), 0.0)
        img = o + g * x + np.where(phi == 0, sg * rng.standard_normal((H, W)), 0.0)
    else:
        img = g * phi + o + sg * rng.standard_normal((H, W))
    return dict(img=f32(img), psf=f32(psf), g=f32(g), o=f32(o), s=f32(sg), per_pixel=per_pixel, k=k,
                camera=1 if emccd else 0)


def gpu_sampler(bdc, P, **kw):
    kw.setdefault("schedule", bdc.BDC_SCHED_CHROMATIC)
    if P["per_pixel"]:
        cam = (P["g"], P["o"], P["s"])
    else:
        cam = (np.float32(P["g"][0, 0]), np.float32(P["o"][0, 0]), np.float32(P["s"][0, 0]))
    H, W = P["img"].shape
    return bdc.Sampler(P["psf"], *cam, height=H, width=W, object_sub=P["k"], camera=P["camera"], **kw)


def oracle_sampler(P, **kw):
    d = lambda a: np.asarray(a, np.float64)
    return oracle.OracleSampler(d(P["img"]), d(P["psf"]), d(P["g"]), d(P["o"]), d(P["s"]), object_sub=P["k"],
                                camera=P["camera"], **kw)


def _asym_psf(s, seed=3):
    rng = np.random.default_rng(seed)
    p = rng.uniform(0.05, 1.0, (s, s))
    p[0, :] *= 3.0
    return p / p.sum()


@pytest.mark.parametrize("k,s,H,W", [(2, 9, 21, 17), (3, 13, 11, 14), (2, 1, 6, 5), (4, 21, 5, 7)])
def test_forward_model_matches_oracle(bdc, k, s, H, W):
    say("forward k=%d s=%d %dx%d" % (k, s, H, W))
    P = make_problem(H, W, k, _asym_psf(s), True, seed=k + s)
    S = gpu_sampler(bdc, P, n_chains=2, seed=1)
    n_groups, sched, _ = S.schedule_info()
    sp = 2 * ((s // 2 + k - 1) // k) + 1
    assert sched == bdc.BDC_SCHED_CHROMATIC and n_groups == k * k * sp * sp
    S.init(P["img"])
    rng = np.random.default_rng(2)
    rho = f32(rng.gamma(2.0, 5.0, (2, k * H, k * W)) + 0.1)
    S.set_rho(rho, np.zeros_like(rho), 0)
    mu = S.mu()
    assert mu.shape == (2, H, W)
    psf = P["psf"].astype(np.float64)
    for c in range(2):
        want = oracle.forward_sub(rho[c].astype(np.float64), psf / psf.sum(), k)
        np.testing.assert_allclose(mu[c], want, rtol=2e-6, atol=1e-6)
    S.close()


@pytest.mark.parametrize("per_pixel", [False, True])
def test_default_initial_state_matches_oracle(bdc, per_pixel):
    """rho0 of cell m in pixel n = max(c_n, 1/2) / k^2 exp(xi_m / 2) (element by element)."""
    P = make_problem(13, 19, 2, synth.gaussian_psf(2.0, 11), per_pixel, seed=61)
    S = gpu_sampler(bdc, P, n_chains=3, seed=0x1234_5678_9ABC, log_step0=-1.25)
    S.init(P["img"])
    rho, ls, t = S.rho()
    O = oracle_sampler(P, n_chains=3, seed=0x1234_5678_9ABC, log_step0=-1.25)
    O.init()
    ro = O.state()[0]
    assert rho.shape == ro.shape == (3, 26, 38)
    err = np.abs(rho - ro) / ro
    say("  max rel err %.3g" % err.max())
    assert err.max() < 5e-6 and np.all(ls == np.float32(-1.25))
    S.close()


def test_loglik_is_on_the_pixel_lattice(bdc):
    P = make_problem(15, 12, 2, synth.gaussian_psf(2.0, 9), True, seed=5)
    S = gpu_sampler(bdc, P, n_chains=1, seed=3)
    S.init(P["img"])
    S.sweep(2)
    ell = S.loglik(0).astype(np.float64)
    mu = S.mu()[0].astype(np.float64)
    want = oracle.loglik(*[P[q].astype(np.float64) for q in ("img", "g", "o", "s")], mu)
    assert ell.shape == (15, 12)
    assert np.max(np.abs(ell - want) / np.maximum(np.abs(want), 1.0)) < 1e-5
    S.close()


def _decision_check(delta_g, acc_g, delta_o, logu_o, acc_o, sabs_o, sel):
    band = 1e-5 * (1.0 + sabs_o[sel])
    clear = np.abs(delta_o[sel] - logu_o[sel]) > band
    err = np.abs(delta_g[sel].astype(np.float64) - delta_o[sel]) / (1.0 + sabs_o[sel])
    bad = clear & (acc_g[sel] != acc_o[sel])
    if bad.any() or err.max() >= 1e-5:
        worst = np.argsort(err)[-5:]
        say("  worst |dDelta|/(1+S):", err[worst], "gpu", delta_g[sel][worst], "oracle", delta_o[sel][worst])
    assert not bad.any(), "decision mismatch outside the tie band"
    return err, int((~clear).sum())


CASES = {
    # (H, W, k, psf, per-pixel maps, EMCCD, photon scale)
    "k2_gauss_maps": (24, 20, 2, lambda: synth.gaussian_psf(2.4, 15), True, False, 1.0),
    "k2_airy_scalar": (22, 26, 2, lambda: synth.airy_psf(1.4, 0.6, 0.0325, 31), False, False, 1.0),
    "k3_gauss_ragged": (17, 13, 3, lambda: synth.gaussian_psf(3.0, 19), True, False, 1.0),
    "k2_emccd_maps": (20, 18, 2, lambda: synth.gaussian_psf(2.4, 15), True, True, 1.0),
    "k2_dim": (18, 16, 2, lambda: synth.gaussian_psf(2.4, 15), True, False, 0.05),
    "k2_small_frame": (3, 5, 2, lambda: synth.gaussian_psf(2.4, 15), True, False, 1.0),
}


@pytest.mark.parametrize("case", list(CASES))
def test_colour_pass_decisions_match_oracle(bdc, case):
    """Single colours from a shared state, then one run of consecutive colours
    (whose accepted moves commit pixel means the later colours read)."""
    H, W, k, mk, pp, em, scale = CASES[case]
    say("object lattice colour pass", case)
    P = make_problem(H, W, k, mk(), pp, seed=11, emccd=em, scale=scale)
    C = 2
    S = gpu_sampler(bdc, P, n_chains=C, seed=99, burn_in=3)
    S.init(P["img"])
    S.sweep(5)
    rho, ls, t = S.rho()
    O = oracle_sampler(P, n_chains=C, seed=99, burn_in=3)
    O.init()
    ng = O.n_groups()
    assert S.schedule_info()[0] == ng
    errs, ties, n = [], 0, 0
    # colours that hold cells of this frame (a frame narrower than the pixel
    # footprint side sp has empty ones)
    sp = int(round(math.sqrt(ng // (k * k))))
    present = sorted({ph * sp * sp + cy * sp + cx for ph in range(k * k) for cy in range(min(H, sp))
                      for cx in range(min(W, sp))})
    for g in sorted(({0, 1, ng // 3, ng // 2, ng - 1} | {present[0], present[-1]}) & set(present)):
        S.set_rho(rho, ls, t)
        dg, ag = S.run_groups(g, g + 1)
        O.set_state(rho.astype(np.float64), ls.astype(np.float64), t)
        do, lo, ao, sa = O.run_groups(t, g, g + 1, with_sabs=True)
        sel = ao != 255
        assert np.array_equal(sel, ag != 255)
        e, kk = _decision_check(dg, ag, do, lo, ao, sa, sel)
        errs.append(e)
        ties += kk
        n += int(sel.sum())
    # a run of colours: later colours read the means earlier ones committed
    g0, g1 = 0, min(ng, 40)
    S.set_rho(rho, ls, t)
    dg, ag = S.run_groups(g0, g1)
    O.set_state(rho.astype(np.float64), ls.astype(np.float64), t)
    do, lo, ao, sa = O.run_groups(t, g0, g1, with_sabs=True)
    sel = ao != 255
    assert np.array_equal(sel, ag != 255)
    tie = sel & (np.abs(do - lo) <= 1e-5 * (1.0 + sa))
    if not tie.any():
        e, _ = _decision_check(dg, ag, do, lo, ao, sa, sel)
        errs.append(e)
        n += int(sel.sum())
        rg = S.rho()[0]
        np.testing.assert_allclose(rg[sel], O.state()[0][sel], rtol=2e-6)
    else:
        say("  a tie in the run of colours: compared single colours only")
    e = np.concatenate(errs)
    say("  decisions %d, ties %d, max |dDelta|/(1+S) %.3g" % (n, ties, e.max()))
    assert n > 0 and e.max() < 1e-5
    S.close()


BLOCK_CASES = {
    # (H, W, k, psf, per-pixel maps, EMCCD, B, groups of one block phase's colours)
    "k2_gauss_B9": (40, 36, 2, lambda: synth.gaussian_psf(2.4, 15), True, False, 9, (0, 60)),
    "k2_gauss_B12_phase1": (40, 36, 2, lambda: synth.gaussian_psf(2.4, 15), True, False, 12, (324 + 100, 324 + 140)),
    "k3_gauss_B8_ragged": (29, 27, 3, lambda: synth.gaussian_psf(3.0, 19), False, False, 8, (2 * 441 + 30, 2 * 441 + 70)),
    "k2_emccd_B9_phase3": (40, 36, 2, lambda: synth.gaussian_psf(2.4, 15), True, True, 9, (3 * 324, 3 * 324 + 50)),
}


@pytest.mark.parametrize("case", list(BLOCK_CASES))
def test_block_phase_decisions_match_oracle(bdc, case):
    """The block scan on the object lattice: one group at a time from a shared
    state (each group's updates are the first of their blocks), then a run of
    groups within one block phase whose decisions commit means the later
    groups of a block read (compared where no tie occurred in the run)."""
    H, W, k, mk, pp, em, B, (g0, g1) = BLOCK_CASES[case]
    say("object lattice block phase", case)
    P = make_problem(H, W, k, mk(), pp, seed=13, emccd=em)
    C = 2
    S = gpu_sampler(bdc, P, n_chains=C, seed=5, burn_in=2, schedule=bdc.BDC_SCHED_BLOCK, block_size=B)
    ng, sched, Bu = S.schedule_info()
    assert sched == bdc.BDC_SCHED_BLOCK and Bu == B
    S.init(P["img"])
    S.sweep(3)
    rho, ls, t = S.rho()
    O = oracle_sampler(P, n_chains=C, seed=5, burn_in=2, schedule=oracle.SCHED_BLOCK, block=B)
    O.init()
    assert O.n_groups() == ng
    errs, n = [], 0
    for g in (g0, g0 + 1, (g0 + g1) // 2, g1 - 1):
        S.set_rho(rho, ls, t)
        dg, ag = S.run_groups(g, g + 1)
        O.set_state(rho.astype(np.float64), ls.astype(np.float64), t)
        do, lo, ao, sa = O.run_groups(t, g, g + 1, with_sabs=True)
        sel = ao != 255
        assert np.array_equal(sel, ag != 255)
        if sel.any():
            e, _ = _decision_check(dg, ag, do, lo, ao, sa, sel)
            errs.append(e)
            n += int(sel.sum())
    S.set_rho(rho, ls, t)
    dg, ag = S.run_groups(g0, g1)
    O.set_state(rho.astype(np.float64), ls.astype(np.float64), t)
    do, lo, ao, sa = O.run_groups(t, g0, g1, with_sabs=True)
    sel = ao != 255
    assert np.array_equal(sel, ag != 255)
    if not (sel & (np.abs(do - lo) <= 1e-5 * (1.0 + sa))).any():
        e, _ = _decision_check(dg, ag, do, lo, ao, sa, sel)
        errs.append(e)
        n += int(sel.sum())
        np.testing.assert_allclose(S.rho()[0][sel], O.state()[0][sel], rtol=2e-6)
    else:
        say("  a tie in the run of groups: compared single groups only")
    e = np.concatenate(errs)
    say("  decisions %d, max |dDelta|/(1+S) %.3g" % (n, e.max()))
    assert n > 0 and e.max() < 1e-5
    S.close()


@pytest.mark.parametrize("k", [2, 3])
def test_one_pixel_of_k2_cells_matches_the_closed_form(bdc, k):
    """PSF a delta on the object lattice: every pixel is its own problem of
    k^2 cells with mu = their sum.  Flat prior: E[rho_i] = E[S] / k^2 and
    E[rho_i^2] = 2 E[S^2] / (k^2 (k^2 + 1)), S ~ L(S) S^(k^2 - 1) by
    quadrature; 32 x 32 replicate pixels give the standard errors."""
    H = W = 32
    G, o, sg, c = 2.0, 100.0, 1.5, 23.4
    K = k * k
    u = np.linspace(math.log(1e-4), math.log(300.0), 40001)
    Sg = np.exp(u)
    lp = oracle.loglik(np.full_like(Sg, o + G * c), G, o, sg, Sg) + K * u
    p = np.exp(lp - lp.max())
    p /= p.sum()
    ES, ES2 = (p * Sg).sum(), (p * Sg * Sg).sum()
    m_q = ES / K
    v_q = 2.0 * ES2 / (K * (K + 1)) - m_q ** 2
    S = bdc.Sampler(f32([[1.0]]), np.float32(G), np.float32(o), np.float32(sg), height=H, width=W, n_chains=2,
                    seed=31, burn_in=600, object_sub=k)
    ng, sched, B = S.schedule_info()
    assert sched == bdc.BDC_SCHED_BLOCK and B == 4 and ng == 4 * K        # automatic: the block scan
    S.init(f32(np.full((H, W), o + G * c)))
    S.sweep(600 + 4000)
    mean, var, n = S.moments(-1)
    assert n == 4000 and mean.shape == (k * H, k * W)
    m_px = _pool(mean.astype(np.float64), k).ravel() / K          # per pixel: mean over its cells
    v_px = _pool(var.astype(np.float64), k).ravel() / K
    zm = (m_px.mean() - m_q) / (m_px.std(ddof=1) / math.sqrt(m_px.size))
    zv = (v_px.mean() - v_q) / (v_px.std(ddof=1) / math.sqrt(v_px.size))
    say("  k %d: mean %.5g (closed form %.5g, z %+.2f), var %.5g (%.5g, z %+.2f)"
        % (k, m_px.mean(), m_q, zm, v_px.mean(), v_q, zv))
    assert abs(zm) < 4.0 and abs(zv) < 4.0
    S.close()


@pytest.mark.parametrize("case", ["gamma_scmos", "flat_emccd"])
def test_moments_match_oracle_run(bdc, case):
    """Posterior means of a 10 x 10 pixel frame on a 20 x 20 object lattice
    (Gaussian PSF on the object lattice) against an oracle run, per cell, within
    the two runs' batch-means standard errors."""
    em = case == "flat_emccd"
    kw = {} if em else dict(prior_kind=oracle.PRIOR_GAMMA, prior_a=2.0, prior_b=0.2)
    say("object-lattice moments vs oracle run:", case)
    P = make_problem(10, 10, 2, synth.gaussian_psf(2.4, 11), False, seed=17, emccd=em)
    burn = 300
    O = oracle_sampler(P, n_chains=2, seed=31, burn_in=burn, **kw)
    O.init()
    O.sweep(burn)
    draws = []
    for _ in range(1200):
        O.sweep(1)
        draws.append(O.state()[0].copy())
    d = np.array(draws)                                   # [n, C, 20, 20]
    mo = d.mean(axis=(0, 1))
    se_o = np.sqrt(np.mean([[[oracle.batch_means_mcse(d[:, c, y, x], 30) ** 2 for x in range(20)]
                             for y in range(20)] for c in range(2)], axis=0) / 2)
    gkw = {} if em else dict(prior_kind=bdc.BDC_PRIOR_GAMMA, prior_a=2.0, prior_b=0.2)
    S = gpu_sampler(bdc, P, n_chains=8, seed=77, burn_in=burn, rhat_block=30, max_sweeps=3300, **gkw)
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


def test_checkpoint_and_exported_draws_are_on_the_object_lattice(bdc):
    """A saved state resumes bit for bit; the thinned draws are the chain's
    object-lattice states at the exported sweeps; a state saved with another
    object_sub is refused."""
    P = make_problem(12, 11, 2, synth.gaussian_psf(2.0, 9), True, seed=9)
    S = gpu_sampler(bdc, P, n_chains=2, seed=5, burn_in=4)
    S.init(P["img"])
    S.set_export(2, 8)
    S.sweep(6)
    state = S.get_state()
    S.sweep(4)
    r1 = S.rho()[0]
    S.set_state(state)
    S.sweep(4)
    r2 = S.rho()[0]
    assert r1.shape == (2, 24, 22) and np.array_equal(r1, r2)
    draws = S.samples()
    assert draws.shape[1:] == (2, 24, 22) and draws.shape[0] == 3          # sweeps 4, 6, 8 (thin 2)
    np.testing.assert_array_equal(S.quantiles([0.0, 1.0])[0], draws.min(axis=(0, 1)))
    P3 = dict(P, k=3)
    T = gpu_sampler(bdc, P3, n_chains=2, seed=5, burn_in=4)
    T.init(P["img"])
    with pytest.raises(bdc.BdcError) as ei:
        T.set_state(state)
    assert ei.value.status == bdc.BDC_EINVAL
    T.close()
    S.close()


def test_pixel_lattice_only_entry_points_refuse_a_finer_object_lattice(bdc):
    P = make_problem(16, 16, 2, synth.gaussian_psf(2.0, 9), True, seed=7)
    for kw in (dict(schedule=bdc.BDC_SCHED_BLOCK9_SERIES), dict(schedule=bdc.BDC_SCHED_BLOCK_SERIES),
               dict(prior_kind=bdc.BDC_PRIOR_DIRICHLET), dict(schedule=bdc.BDC_SCHED_BLOCK, block_size=3)):
        with pytest.raises(bdc.BdcError) as ei:
            gpu_sampler(bdc, P, **kw)
        assert ei.value.status == bdc.BDC_EINVAL
    S = gpu_sampler(bdc, P, n_chains=1, seed=1)
    S.init(P["img"])
    for call in (lambda: S.richardson_lucy(3), lambda: S.init_rl(3), lambda: bdc.Batch([S]),
                 lambda: S.set_schedule(bdc.BDC_SCHED_BLOCK_SERIES, 0), lambda: S.training_targets()):
        with pytest.raises(bdc.BdcError) as ei:
            call()
        assert ei.value.status in (bdc.BDC_EINVAL, bdc.BDC_ESTATE)
    ms, best = S.autotune([0, 2, -5, -1005], 1)               # footprint side 5: blocks of >= 4 pixels
    assert best == 0 and all(math.isinf(m) for m in ms[1:])
    assert S.schedule_info()[1] == bdc.BDC_SCHED_CHROMATIC
    S.sweep(3)                                    # still runs after the refusals
    S.close()
