"""Richardson-Lucy on the GPU against the FP64 reference (oracle/rl.py): the
paper's baseline deconvolution, and the warm start of the sampler from it."""

import numpy as np
import pytest

import oracle
from oracle import rl
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


CASES = {
    "airy31_ragged_maps": (70, 66, lambda: synth.airy_psf(1.4, 0.6, 0.065, 31), True),
    "gauss11_scalar": (64, 64, lambda: synth.gaussian_psf(1.5, 11), False),
    "asym7_small": (9, 40, None, True),
}


@pytest.mark.parametrize("case", list(CASES))
def test_richardson_lucy_matches_reference(bdc, case):
    H, W, mk, pp = CASES[case]
    say("Richardson-Lucy:", case)
    rng = np.random.default_rng(H + W)
    if mk is None:
        psf = rng.uniform(0.05, 1.0, (7, 7))
        psf[0] *= 3.0
        psf /= psf.sum()
    else:
        psf = mk()
    truth = np.full((H, W), 3.0)
    synth.add_beads(truth, rng, max(1, H * W // 80))
    synth.add_filaments(truth, rng, max(1, H // 20))
    cam = synth.scmos_maps(rng, H, W) if pp else synth.scalar_camera()
    img = synth.simulate_frame(truth, psf, cam, rng).astype(np.float32)
    g, o, s = [np.asarray(a, np.float32) for a in cam.maps(H, W)]
    if pp:
        S = bdc.Sampler(psf.astype(np.float32), g, o, s, height=H, width=W)
    else:
        S = bdc.Sampler(psf.astype(np.float32), np.float32(2.0), np.float32(100.0), np.float32(1.5), height=H, width=W)
    S.init(img)
    d = rl.photon_image(img.astype(np.float64), g.astype(np.float64), o.astype(np.float64))
    p64 = psf.astype(np.float32).astype(np.float64)
    norm = rl._corr(np.ones_like(d), p64 / p64.sum())
    for n_iter, tol in ((1, 2e-6), (10, 2e-5), (50, 2e-4)):
        got = S.richardson_lucy(n_iter).astype(np.float64)
        want = rl.richardson_lucy(d, p64, n_iter)
        err = np.abs(got - want).max() / want.max()
        say("  %d iterations: max |gpu - ref| / max ref = %.3g" % (n_iter, err))
        assert err < tol
        assert (got * norm).sum() == pytest.approx(d.sum(), rel=1e-5)
    S.close()


def test_rl_warm_start_of_the_chains(bdc):
    say("RL warm start")
    fr = synth.frame_beads_segments(48, seed=7, n_prims=10)
    H, W = fr.image.shape
    img = fr.image.astype(np.float32)
    C, seed = 3, 0xABCDEF
    S = bdc.Sampler(fr.psf.astype(np.float32), np.float32(2.0), np.float32(100.0), np.float32(1.5), height=H,
                    width=W, n_chains=C, seed=seed, log_step0=-1.0)
    S.init(img)
    S.sweep(3)
    est = S.richardson_lucy(20).astype(np.float64)
    S.init_rl(20)
    rho, ls, t = S.rho()
    assert t == 0 and np.all(ls == np.float32(-1.0))
    for c in range(C):
        xi = np.array([[oracle.normal(seed, y * W + x, 0, c, 2) for x in range(W)] for y in range(H)])
        want = np.maximum(est, 1e-3) * np.exp(0.5 * xi)
        np.testing.assert_allclose(rho[c], want, rtol=5e-6)
    S.sweep(5)
    assert np.all(S.rho()[0] > 0)
    S.close()
