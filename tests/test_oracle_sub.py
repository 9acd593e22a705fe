"""CPU pins of the oracle's finer object lattice (Methods, Image Formation
Model, Eqs. 1-2: mu_n integrates the blurred object over pixel n; here the
object is discretised on k x k cells per camera pixel and the PSF is sampled
on that lattice).

Pinned against: SciPy's 2-D convolution followed by k x k sum-pooling (the
forward model), k = 1 reducing to the pixel-lattice oracle, brute-force
coverage and disjoint pixel footprints of the scan's groups, Delta against
two full log-posterior evaluations (sCMOS and EMCCD readings), and the
one-pixel posterior of k^2 cells in closed form: with a flat prior the sum
S of the cells has density proportional to L(S) S^(k^2 - 1) and the cells
given S are S times a flat Dirichlet, so E[rho_i] = E[S] / k^2 and
E[rho_i^2] = 2 E[S^2] / (k^2 (k^2 + 1)).
"""

import math

import numpy as np
import pytest
from scipy import signal

import oracle
from paper_2411_00991_amd import synth


def _pool(a, k):
    H, W = a.shape[0] // k, a.shape[1] // k
    return a.reshape(H, k, W, k).sum(axis=(1, 3))


@pytest.mark.parametrize("k,s,H,W", [(2, 7, 9, 11), (3, 9, 5, 7), (2, 1, 4, 3), (4, 11, 3, 5)])
def test_forward_sub_is_convolution_then_pixel_integration(k, s, H, W):
    rng = np.random.default_rng(k * 100 + s)
    rho = rng.gamma(2.0, 3.0, (k * H, k * W))
    psf = rng.uniform(0.0, 1.0, (s, s))
    psf[0, :] *= 4.0                                  # asymmetric: a flipped kernel would show
    want = _pool(signal.convolve2d(rho, psf, mode="same", boundary="fill", fillvalue=0.0), k)
    np.testing.assert_allclose(oracle.forward_sub(rho, psf, k), want, rtol=1e-13, atol=1e-12)


def test_forward_sub_with_k_1_is_the_pixel_lattice_forward():
    rng = np.random.default_rng(5)
    rho = rng.gamma(2.0, 3.0, (13, 17))
    psf = rng.uniform(0.0, 1.0, (7, 7))
    assert np.array_equal(oracle.forward_sub(rho, psf, 1), oracle.forward(rho, psf))


@pytest.mark.parametrize("k,s,H,W,B", [(2, 7, 11, 9, 0), (3, 9, 7, 8, 0), (2, 3, 5, 5, 0), (2, 1, 3, 4, 0),
                                       (4, 15, 6, 5, 0), (2, 7, 11, 9, 4), (2, 7, 13, 12, 5), (3, 9, 10, 11, 5),
                                       (2, 1, 5, 4, 1), (2, 13, 17, 15, 6)])
def test_object_scan_covers_every_cell_once_with_disjoint_pixel_footprints(k, s, H, W, B):
    """The pixels a cell's light reaches (the PSF's support moved to the cell,
    mapped to pixels) are pairwise disjoint within each group, and every cell
    is in exactly one group (pixel-chromatic scan, B = 0, and the block scan
    with B x B-pixel blocks)."""
    img = np.full((H, W), 100.0)
    kw = dict(schedule=oracle.SCHED_BLOCK, block=B) if B else {}
    S = oracle.OracleSampler(img, np.ones((s, s)), 2.0, 100.0, 1.5, object_sub=k, **kw)
    Ho, Wo, r = k * H, k * W, s // 2
    reach = {}
    for m in range(Ho * Wo):
        y, x = divmod(m, Wo)
        reach[m] = {(cy // k, cx // k) for cy in range(max(0, y - r), min(Ho, y + r + 1))
                    for cx in range(max(0, x - r), min(Wo, x + r + 1))}
    seen = np.zeros(Ho * Wo, int)
    for g in range(S.n_groups()):
        cells = S.group(g)
        seen[cells] += 1
        taken = set()
        for m in cells:
            assert not (reach[int(m)] & taken), "two cells of one group reach the same pixel"
            taken |= reach[int(m)]
    assert np.all(seen == 1)


@pytest.mark.parametrize("camera,B", [(0, 0), (1, 0), (0, 4)])
def test_cell_delta_equals_difference_of_full_log_posteriors(camera, B):
    k, s, H, W = 2, 7, 8, 9
    rng = np.random.default_rng(11 + camera)
    psf = synth.gaussian_psf(1.6, s)
    cam = synth.scmos_maps(rng, H, W)
    truth = rng.gamma(2.0, 10.0, (k * H, k * W)) + 1.0
    mu = _pool(signal.convolve2d(truth, psf, mode="same"), k)
    phi = rng.poisson(mu)
    g, o, sg = cam.maps(H, W)
    if camera:
        x = np.where(phi > 0, rng.gamma(np.maximum(phi, 1), 1.0), 0.0)
        img = o + g * x + np.where(phi == 0, sg * rng.standard_normal((H, W)), 0.0)
    else:
        img = g * phi + o + sg * rng.standard_normal((H, W))
    seed, t = 4321, 3
    kw = dict(n_chains=2, seed=seed, prior_kind=oracle.PRIOR_GAMMA, prior_a=1.5, prior_b=0.01, camera=camera,
              object_sub=k, **(dict(schedule=oracle.SCHED_BLOCK, block=B) if B else {}))
    S = oracle.OracleSampler(img, psf, g, o, sg, burn_in=10, **kw)
    S.init()
    rho0, ls0, _, _ = S.state()
    assert rho0.shape == (2, k * H, k * W)
    R = oracle.OracleSampler(img, psf, g, o, sg, **kw)
    R.init()
    Wo = k * W
    for gidx in (0, 5, S.n_groups() - 1):
        S.set_state(rho0, ls0, t)
        delta, logu, acc = S.run_groups(t, gidx, gidx + 1)
        cells = S.group(gidx)
        assert np.count_nonzero(acc != 255) == 2 * len(cells)
        for ch in range(2):
            R.set_state(rho0, ls0, t)
            lp0 = R.log_posterior(ch)
            for m in cells[:5]:
                y, x = divmod(int(m), Wo)
                xi = oracle.normal(seed, int(m), t, ch, 0)
                rp = rho0[ch, y, x] * math.exp(math.exp(ls0[ch, y, x]) * xi)
                r1 = rho0.copy()
                r1[ch, y, x] = rp
                R.set_state(r1, ls0, t)
                want = R.log_posterior(ch) - lp0 + math.log(rp / rho0[ch, y, x])
                assert delta[ch, y, x] == pytest.approx(want, abs=1e-9)
                assert acc[ch, y, x] == int(logu[ch, y, x] < delta[ch, y, x])


def test_committed_means_follow_the_state():
    """After a sweep the incrementally committed pixel means equal the
    forward model of the new state."""
    k, s, H, W = 3, 5, 6, 7
    rng = np.random.default_rng(2)
    psf = synth.gaussian_psf(1.2, s)
    img = 100.0 + 2.0 * rng.poisson(20.0, (H, W))
    S = oracle.OracleSampler(img, psf, 2.0, 100.0, 1.5, n_chains=2, seed=3, object_sub=k)
    S.init()
    S.run_groups(0, 0, S.n_groups())
    rho, _, mu, _ = S.state()
    for ch in range(2):
        np.testing.assert_allclose(mu[ch], oracle.forward_sub(rho[ch], psf / psf.sum(), k), rtol=1e-10)


@pytest.mark.parametrize("k", [2, 3])
def test_one_pixel_of_k2_cells_matches_the_closed_form(k):
    """One pixel, PSF a delta on the object lattice (mu = sum of the pixel's
    k^2 cells), flat prior: E[rho_i] = E[S] / k^2 and
    E[rho_i^2] = 2 E[S^2] / (k^2 (k^2 + 1)) with S ~ L(S) S^(k^2 - 1) by quadrature."""
    w, G, o, sig = 100.0 + 2.0 * 23.4, 2.0, 100.0, 1.5
    K = k * k
    u = np.linspace(math.log(1e-4), math.log(300.0), 40001)
    Sg = np.exp(u)
    lp = oracle.loglik(np.full_like(Sg, w), G, o, sig, Sg) + K * u       # density of log S
    p = np.exp(lp - lp.max())
    p /= p.sum()
    ES, ES2 = (p * Sg).sum(), (p * Sg * Sg).sum()
    mean_i = ES / K
    var_i = 2.0 * ES2 / (K * (K + 1)) - mean_i ** 2
    S = oracle.OracleSampler(np.array([[w]]), np.array([[1.0]]), G, o, sig, n_chains=4, seed=29, burn_in=600,
                             object_sub=k)
    assert S.n_groups() == K
    S.init()
    S.sweep(600)
    draws = []
    for _ in range(12000):
        S.sweep(1)
        draws.append(S.state()[0].copy())
    d = np.array(draws)                                                   # [n, C, k, k]
    n, C = d.shape[:2]
    flat = d.reshape(n, C, K)
    z = []
    for i in range(K):
        se = math.sqrt(np.mean([oracle.batch_means_mcse(flat[:, c, i], 40) ** 2 for c in range(C)]) / C)
        z.append((flat[:, :, i].mean() - mean_i) / se)
    assert np.all(np.abs(z) < 4.0), (z, mean_i)
    np.testing.assert_allclose(flat.reshape(-1, K).var(axis=0, ddof=1), var_i, rtol=0.12)


def test_finer_lattice_refuses_nine_phase_scans_small_blocks_and_the_chunk_prior():
    """Block side in pixels at least sp - 1 (sp = 3 for a 5 x 5 PSF on a lattice
    twice as fine): B = 1 would put same-group cells of neighbouring
    same-phase blocks within one pixel footprint."""
    img = np.full((8, 8), 120.0)
    psf = np.ones((5, 5))
    for kw in (dict(schedule=oracle.SCHED_BLOCK, block=1), dict(schedule=oracle.SCHED_BLOCK9, block=3),
               dict(prior_kind=oracle.PRIOR_DIRICHLET, schedule=oracle.SCHED_BLOCK, block=3)):
        with pytest.raises(ValueError):
            oracle.OracleSampler(img, psf, 2.0, 100.0, 1.5, object_sub=2, **kw)
    S = oracle.OracleSampler(img, psf, 2.0, 100.0, 1.5, object_sub=2, schedule=oracle.SCHED_BLOCK, block=2)
    assert S.n_groups() == 4 * 4 * 9
    with pytest.raises(ValueError):
        oracle.OracleSampler(img, psf, 2.0, 100.0, 1.5, object_sub=5)
