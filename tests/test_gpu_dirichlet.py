"""The Dirichlet-OTF prior (Methods, Prior, Eqs. 7-8) on the GPU, read per
chunk (the B x B blocks of the block-phase scan), against the FP64 oracle:
accept decisions and Delta of block-phase groups from a shared state (tie band
1e-5 (1 + S), S including the prior's terms, widened by Delta's sensitivity
to the FP32 rounding of the proposal), the log-posterior trace with
every chunk's log prior, and the 2-pixel posterior by quadrature.
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


# Ranges of groups run the chunk's updates in sequence (the spectrum is updated
# in LDS after every accepted move).  For even chunk sides the Nyquist
# components of a chunk's spectrum are real and can pass close to zero, where
# the Dirichlet's log density (alpha_k < 1) is singular: there the FP32 state
# of the GPU and the FP64 state of the oracle, a few ulp apart after some
# accepted moves, give measurably different Deltas although both are right for
# their own state.  Even sides are therefore compared one group at a time from
# the common state (each group's updates are the first of their blocks).
CASES = {
    # name: (H, W, psf, per-pixel maps, B, groups: a range (g0, g1) or a list of single groups)
    "gauss7_B7_edges": (48, 40, lambda: synth.gaussian_psf(1.2, 7), True, 7, (0, 49)),
    "gauss7_B7_scalar": (45, 52, lambda: synth.gaussian_psf(1.2, 7), False, 7, (3 * 49, 3 * 49 + 30)),
    "airy31_B31_part": (70, 66, lambda: synth.airy_psf(1.4, 0.6, 0.065, 31), True, 31, (961 + 300, 961 + 330)),
    "gauss7_B6_single": (45, 52, lambda: synth.gaussian_psf(1.2, 7), False, 6, [0, 8, 24, 49 + 3, 98 + 16, 147 + 22,
                                                                              147 + 40]),
    "gauss7_B6_maps_single": (45, 52, lambda: synth.gaussian_psf(1.2, 7), True, 6, [5, 49 + 29, 98 + 35, 147 + 9]),
    "gauss7_B7_maps_single": (48, 40, lambda: synth.gaussian_psf(1.2, 7), True, 7, [0, 8, 24, 48, 49 + 3, 98 + 16,
                                                                              147 + 22, 147 + 48]),
}
FLAT_CONTROLS = {"gauss7_B6_single"}


# The EMCCD reading (an EMCCD frame) under the chunk prior, one group at a
# time for odd sides too: on oracle chains of these frames, rounding the
# committed state to FP32 between the groups of a range moves later Deltas by
# up to 1e-4 (sCMOS frames alike), the same singular sensitivity as above.
EMCCD_CASES = {"gauss7_B7_maps_single", "gauss7_B6_maps_single"}


@pytest.mark.parametrize("case,flat,emccd", [(c, False, False) for c in CASES]
                         + [(c, True, False) for c in sorted(FLAT_CONTROLS)]
                         + [(c, False, True) for c in sorted(EMCCD_CASES)])
def test_dirichlet_decisions_match_oracle(bdc, case, flat, emccd):
    H, W, mk, pp, B, groups = CASES[case]
    say("Dirichlet-OTF prior decisions:", case, "(flat-prior control)" if flat else "", "(EMCCD)" if emccd else "")
    if emccd:
        from test_gpu_emccd import make_problem as make_emccd_problem
        P = make_emccd_problem(H, W, mk(), pp, seed=81)
    else:
        P = make_problem(H, W, mk(), pp, seed=81)
    cam = {"camera": 1} if emccd else {}
    s = P["psf"].shape[0]
    C = 2
    kind_g = bdc.BDC_PRIOR_FLAT if flat else bdc.BDC_PRIOR_DIRICHLET
    kind_o = oracle.PRIOR_FLAT if flat else oracle.PRIOR_DIRICHLET
    S = gpu_sampler(bdc, P, n_chains=C, seed=55, burn_in=2, schedule=bdc.BDC_SCHED_BLOCK, block_size=B,
                    prior_kind=kind_g, **cam)
    n_groups, sched, Bu = S.schedule_info()
    assert sched == bdc.BDC_SCHED_BLOCK and Bu == B
    S.init(P["img"])
    S.sweep(3)
    rho, ls, t = S.rho()
    O = oracle_sampler(P, n_chains=C, seed=55, burn_in=2, schedule=oracle.SCHED_BLOCK, block=B,
                       prior_kind=kind_o, **cam)
    O.init()
    ranges = [groups] if isinstance(groups, tuple) else [(g, g + 1) for g in groups]
    shp = (C, H, W)
    dg, do, lu, sa = [np.zeros(shp) for _ in range(4)]
    ag = np.full(shp, 255, np.uint8)
    ao = np.full(shp, 255, np.uint8)
    rg = np.zeros(shp, np.float32)
    ro = np.zeros(shp)
    for g0, g1 in ranges:
        S.set_rho(rho, ls, t)
        dgi, agi = S.run_groups(g0, g1)
        O.set_state(rho.astype(np.float64), ls.astype(np.float64), t)
        doi, lui, aoi, sai = O.run_groups(t, g0, g1, with_sabs=True)
        m = aoi != 255
        assert m.sum() > 0 and np.array_equal(m, agi != 255)
        dg[m], ag[m], do[m], lu[m], ao[m], sa[m] = dgi[m], agi[m], doi[m], lui[m], aoi[m], sai[m]
        rg[m] = S.rho()[0][m]
        ro[m] = O.state()[0][m]
    sel = ao != 255
    # Delta's sensitivity to the FP32 rounding of the proposal: the GPU draws
    # rho' = rho exp(h) in FP32, h = step * xi, so rho' carries a relative
    # rounding of a few ulp times (1 + |h|) against the oracle's FP64 draw,
    # and the chunk prior changes by sum_k (alpha_k - 1) d log|F_k| per unit
    # of rho', at most sum_k |alpha_k - 1| / |F'_k| + (K - 1) K / S'
    sens = np.zeros_like(sa)
    psf64 = P["psf"].astype(np.float64)
    for c, y, x in zip(*np.nonzero(sel)):
        y0, x0 = (y // B) * B, (x // B) * B
        th, tw = min(B, H - y0), min(B, W - x0)
        al = oracle.dirichlet_alpha(psf64, th, tw)
        chunk = rho[c, y0:y0 + th, x0:x0 + tw].astype(np.float64).copy()
        m = int(y * W + x)
        h = np.exp(float(ls[c, y, x])) * oracle.normal(55, m, t, c, 0)
        rp = chunk[y - y0, x - x0] * np.exp(h)
        chunk[y - y0, x - x0] = rp
        Fm = np.abs(np.fft.fft2(chunk))
        sens[c, y, x] = 0.0 if flat else (1.0 + abs(h)) * abs(rp) * ((np.abs(al - 1.0) / Fm).sum() + (al.size - 1) * al.size / Fm.sum())
    band = 1e-5 * (1.0 + sa) + 1e-6 * sens
    tie = sel & (np.abs(do - lu) <= band)
    keep = sel.copy()
    for c, y, x in zip(*np.nonzero(tie)):
        by, bx = y // B, x // B
        g_tie = ((y - by * B) % s) * s + ((x - bx * B) % s)
        yy, xx = np.mgrid[by * B:min((by + 1) * B, H), bx * B:min((bx + 1) * B, W)]
        later = ((yy - by * B) % s) * s + ((xx - bx * B) % s) >= g_tie
        keep[c, yy[later], xx[later]] = False
    err = np.abs(dg[keep].astype(np.float64) - do[keep]) / band[keep] * 1e-5
    if not np.array_equal(ag[keep], ao[keep]) or err.max() >= 1e-5:
        w = np.argsort(err)[-6:]
        kc, ky_, kx_ = np.nonzero(keep)
        for i in w:
            c, y, x = kc[i], ky_[i], kx_[i]
            say("  worst: chain %d pixel (%d, %d) block-local (%d, %d) acc %d gpu %.7g oracle %.7g S %.4g "
                "band %.3g rho %.5g" % (c, y, x, y % B, x % B, ao[c, y, x], dg[c, y, x], do[c, y, x], sa[c, y, x],
                                      band[c, y, x], rho[c, y, x]))
    assert np.array_equal(ag[keep], ao[keep]), "decision mismatch outside the tie band"
    say("  decisions %d (ties %d), accepted %d, max |dDelta| / band %.3g" % (
        keep.sum(), tie.sum(), int(ao[keep].sum()), err.max()))
    assert err.max() < 1e-5
    np.testing.assert_allclose(rg[keep], ro[keep], rtol=2e-6)
    S.close()


def test_dirichlet_trace_includes_every_chunk_prior(bdc):
    say("Dirichlet-OTF prior: log-posterior trace")
    P = make_problem(33, 29, synth.gaussian_psf(1.2, 7), True, seed=82)
    S = gpu_sampler(bdc, P, n_chains=2, seed=3, schedule=bdc.BDC_SCHED_BLOCK, block_size=7,
                    prior_kind=bdc.BDC_PRIOR_DIRICHLET)
    S.init(P["img"])
    S.sweep(4)
    tr = S.trace()
    rho, ls, t = S.rho()
    O = oracle_sampler(P, n_chains=2, seed=3, schedule=oracle.SCHED_BLOCK, block=7, prior_kind=oracle.PRIOR_DIRICHLET)
    O.init()
    O.set_state(rho.astype(np.float64), ls.astype(np.float64), t)
    for c in range(2):
        say("  chain %d: gpu %.6f oracle %.6f" % (c, tr[-1, c], O.log_posterior(c)))
        assert tr[-1, c] == pytest.approx(O.log_posterior(c), rel=2e-6)
    S.close()


def test_dirichlet_two_pixel_posterior_matches_quadrature(bdc):
    from test_oracle_pins import two_pixel_dirichlet_posterior
    say("Dirichlet-OTF prior: two-pixel quadrature")
    w = np.array([140.0, 118.0])
    row = [0.05, 0.9, 0.05]
    mean, var = two_pixel_dirichlet_posterior(w, 2.0, 100.0, 1.5, row)
    psf = np.zeros((3, 3), np.float32)
    psf[1] = row
    S = bdc.Sampler(psf, np.float32(2.0), np.float32(100.0), np.float32(1.5), height=1, width=2, n_chains=64,
                    seed=6, burn_in=500, rhat_block=50, max_sweeps=5000, schedule=bdc.BDC_SCHED_BLOCK,
                    prior_kind=bdc.BDC_PRIOR_DIRICHLET)
    S.init(f32(w[None, :]))
    S.sweep(5000)
    m, v, n = S.moments()
    se = S.mcse()
    z = (m[0] - mean) / se[0]
    say("  means", m[0], mean, "z", z, "var", v[0], var)
    assert np.all(np.abs(z) < 4.0)
    np.testing.assert_allclose(v[0], var, rtol=0.05)
    S.close()


def test_dirichlet_prior_validation(bdc):
    say("Dirichlet-OTF prior: configurations it refuses")
    psf = f32(synth.gaussian_psf(1.2, 7))
    one = np.float32
    with pytest.raises(bdc.BdcError) as ei:
        bdc.Sampler(psf, one(2.0), one(100.0), one(1.5), height=32, width=32, schedule=bdc.BDC_SCHED_BLOCK_SERIES,
                    prior_kind=bdc.BDC_PRIOR_DIRICHLET)
    assert ei.value.status == bdc.BDC_EINVAL
    with pytest.raises(bdc.BdcError) as ei:
        bdc.Sampler(psf, one(2.0), one(100.0), one(1.5), height=32, width=32, schedule=bdc.BDC_SCHED_BLOCK,
                    block_size=14, prior_kind=bdc.BDC_PRIOR_DIRICHLET)
    assert ei.value.status == bdc.BDC_EINVAL
    S = bdc.Sampler(psf, one(2.0), one(100.0), one(1.5), height=32, width=32, prior_kind=bdc.BDC_PRIOR_DIRICHLET)
    assert S.schedule_info()[1:] == (bdc.BDC_SCHED_BLOCK, 7)
    S.init(np.full((32, 32), 120.0, np.float32))
    S.set_block_proposal(np.zeros((32, 32), np.float32), np.ones((32, 32), np.float32))
    with pytest.raises(bdc.BdcError) as ei:
        S.block_move(1)
    assert ei.value.status == bdc.BDC_EINVAL
    S.close()
