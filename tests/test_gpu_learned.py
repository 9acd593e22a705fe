"""The learned part on the GPU, through the C ABI, against the FP64 oracles.

* the BF16 matrix-core GEMM tile against exact products of the BF16 inputs;
* U-Net forward and gradients against oracle/unet.py (BF16 tolerances below);
* the Adam step against its definition at step 1;
* the block independence move: decisions of one block colour from a shared
  state against oracle.c (tie band as for single-pixel updates), and block
  moves alone against the closed-form and quadrature posteriors;
* the learned warm start against its definition with a zero network.

BF16 tolerance: BF16 keeps 8 significant bits (unit roundoff 2^-9 ~ 2e-3).
Each layer rounds its weights and its input activations once, so a layer's
output carries ~2 such relative errors of random sign per product; through
the ~L = 4 (levels - 1) + 3 layers of a U-Net path the relative error of the
output grows like 2e-3 * sqrt(2 L) ~ 1e-2 in the rms.  Outputs are compared in
relative L2 norm at 3e-2 (3x that estimate); gradients, which pass through
the chain twice (forward activations and backward signals, also BF16), at
6e-2 per layer tensor.
"""

import math
import os
import sys

import numpy as np
import pytest

import oracle
from oracle import unet as U
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


def bf16_bits(x):
    """Round-to-nearest-even BF16 patterns of float32 values (test side)."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    return r


def bits_to_f64(b):
    return (np.asarray(b, np.uint32) << 16).view(np.float32).astype(np.float64)


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


# ---------------------------------------------------------------------------
# Matrix-core tile
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("M,N,K", [(200, 48, 72), (128, 128, 32), (33, 130, 264), (1000, 256, 2304), (7, 9, 8)])
def test_gemm_tile_matches_exact_products(bdc, M, N, K):
    say("gemm %dx%dx%d" % (M, N, K))
    rng = np.random.default_rng(M + N + K)
    a = bf16_bits(rng.standard_normal((M, K)))
    b = bf16_bits(rng.standard_normal((N, K)))
    c = bdc.bdc_debug_gemm_bf16(a, b)
    A, B = bits_to_f64(a), bits_to_f64(b)
    ref = A @ B.T
    scale = np.abs(A) @ np.abs(B).T
    err = np.abs(c - ref) / (scale + 1e-30)
    say("  max |err| / sum|products| = %.3g" % err.max())
    # products of BF16 values are exact in FP32; only the FP32 sum rounds
    assert err.max() < 4 * K * 2.0 ** -24 + 1e-7


# ---------------------------------------------------------------------------
# U-Net forward / backward
# ---------------------------------------------------------------------------

def _params(levels, base, seed):
    r = np.random.default_rng(seed)
    p = U.init_params(levels, base, seed)
    p += 0.02 * r.standard_normal(p.size)
    return p


@pytest.mark.parametrize("levels,base", [(3, 8), (4, 32)])
def test_param_count_matches_oracle(bdc, levels, base):
    net = bdc.UNet(levels, base, max_pixels=1 << 12)
    assert net.n_params == U.param_count(levels, base)
    net.close()


@pytest.mark.parametrize("levels,base,B,H,W", [(4, 16, 2, 32, 32), (4, 32, 1, 64, 48), (3, 8, 3, 16, 24)])
def test_unet_forward_matches_oracle(bdc, levels, base, B, H, W):
    say("unet forward L=%d base=%d %dx%dx%d" % (levels, base, B, H, W))
    rng = np.random.default_rng(7)
    p = _params(levels, base, 3)
    x = np.abs(rng.gamma(2.0, 0.5, (B, H, W))).astype(np.float32)
    net = bdc.UNet(levels, base, max_pixels=B * H * W)
    net.set_params(f32(p))
    out = net.forward(x)
    ref = U.forward(f32(p).astype(np.float64), x.astype(np.float64), levels, base)
    e = [rel_l2(out[..., k], ref[..., k]) for k in range(2)]
    say("  rel L2 error (m, s): %.3g %.3g" % tuple(e))
    assert max(e) < 3e-2
    # element by element: BF16 rounding scatters each output by about 1e-2 of
    # the output scale; a wrong tile seam or halo moves whole pixels by O(1)
    for k in range(2):
        rms = np.sqrt(np.mean(ref[..., k] ** 2))
        worst = np.abs(out[..., k] - ref[..., k]).max() / rms
        say("  max |gpu - oracle| / rms, output %d: %.3g" % (k, worst))
        assert worst < 0.15
    np.testing.assert_array_equal(net.get_params(), f32(p))
    net.close()


@pytest.mark.parametrize("levels,base,B,H,W", [(3, 8, 2, 16, 16), (3, 32, 2, 32, 32), (4, 32, 2, 64, 64)])
def test_unet_gradients_match_oracle(bdc, levels, base, B, H, W):
    say("unet gradients L=%d base=%d %dx%dx%d" % (levels, base, B, H, W))
    rng = np.random.default_rng(8)
    p = f32(_params(levels, base, 4))
    x = np.abs(rng.gamma(2.0, 0.5, (B, H, W))).astype(np.float32)
    tgt = f32(rng.standard_normal((B, H, W, 2)))
    net = bdc.UNet(levels, base, max_pixels=B * H * W, training=True)
    net.set_params(p)
    loss, g = net.gradients(x, tgt)
    loss_o, g_o = U.loss_and_grads(p.astype(np.float64), x.astype(np.float64), tgt.astype(np.float64), levels, base)
    say("  loss gpu %.6g oracle %.6g" % (loss, loss_o))
    assert loss == pytest.approx(loss_o, rel=2e-2)
    k = 0
    worst = 0.0
    worst_el = 0.0
    for name, kind, ci, co in U.layer_specs(levels, base):
        nw = {"conv": co * 9 * ci, "up": 4 * co * ci, "head": 2 * ci}[kind]
        for part, n in (("W", nw), ("b", co)):
            e = rel_l2(g[k:k + n], g_o[k:k + n])
            worst = max(worst, e)
            if e >= 6e-2:
                say("  %s.%s rel L2 %.3g" % (name, part, e))
            assert e < 6e-2, (name, part, e)
            # element by element, against the tensor's scale: a missing, doubled
            # or misplaced split-K partial leaves an entry off by its whole value,
            # >= 1 rms for the entries that carry the tensor; BF16 rounding
            # scatters entries by ~6e-2 rms, whose maximum over thousands of
            # entries reaches ~0.5 rms
            ref = g_o[k:k + n]
            el = np.abs(g[k:k + n] - ref).max() / max(np.sqrt(np.mean(ref ** 2)), 1e-30)
            worst_el = max(worst_el, el)
            assert el < 1.0, (name, part, el)
            k += n
    say("  worst per-tensor rel L2 %.3g, worst entry / tensor rms %.3g" % (worst, worst_el))
    net.close()


def test_adam_step_matches_definition_at_step_one(bdc):
    levels, base, B, H, W = 3, 8, 2, 16, 16
    rng = np.random.default_rng(9)
    p = f32(_params(levels, base, 5))
    x = np.abs(rng.gamma(2.0, 0.5, (B, H, W))).astype(np.float32)
    tgt = f32(rng.standard_normal((B, H, W, 2)))
    net = bdc.UNet(levels, base, max_pixels=B * H * W, training=True)
    net.set_params(p)
    _, g = net.gradients(x, tgt)
    lr = 1e-3
    net.train_step(x, tgt, lr)
    p1 = net.get_params()
    # step 1: m_hat = g and v_hat = g^2, so the update is lr * g / (|g| + eps)
    expect = p.astype(np.float64) - lr * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(p1, expect, rtol=1e-6, atol=2e-6 * lr)
    # and a few more steps on the same batch lower the loss
    l0 = net.gradients(x, tgt)[0]
    for _ in range(40):
        net.train_step(x, tgt, 3e-3, want_loss=False)
    l1 = net.gradients(x, tgt)[0]
    say("  loss %.4g -> %.4g after 41 steps" % (l0, l1))
    assert l1 < 0.7 * l0
    net.close()


# ---------------------------------------------------------------------------
# Block independence move
# ---------------------------------------------------------------------------

def _frame(H, W, psf, seed):
    rng = np.random.default_rng(seed)
    truth = np.full((H, W), 3.0)
    synth.add_beads(truth, rng, max(1, H * W // 80), scale=40.0)
    synth.add_filaments(truth, rng, max(1, H // 24), scale=25.0)
    cam = synth.scmos_maps(rng, H, W)
    img = synth.simulate_frame(truth, psf, cam, rng)
    g, o, s = cam.maps(H, W)
    return f32(img), f32(psf), f32(g), f32(o), f32(s), truth


@pytest.mark.parametrize("H,W,psf_kind,colours,width,beta", [(70, 52, "gauss11", (0, 1, 3), 0.08, 1.0),
                                                              (80, 96, "airy31", (0, 4, 8), 0.08, 1.0),
                                                              (64, 64, "gauss11", (0, 2), 0.7, 1.0),
                                                              (80, 96, "airy31", (1, 5), 0.5, 0.2)])
def test_block_colour_decisions_match_oracle(bdc, H, W, psf_kind, colours, width, beta):
    """width 0.7: proposals far from the current state (likelihood ratios of
    many orders of magnitude per pixel, both ways); beta 0.2: the
    autoregressive proposal around the reference."""
    say("block colour decisions %dx%d %s width %.2f beta %.2f" % (H, W, psf_kind, width, beta))
    psf = synth.gaussian_psf(1.5, 11) if psf_kind == "gauss11" else synth.airy_psf(1.4, 0.6, 0.065, 31)
    img, psf, g, o, s, truth = _frame(H, W, psf, seed=31)
    C, seed = 2, 77
    S = bdc.Sampler(psf, g, o, s, height=H, width=W, n_chains=C, seed=seed, burn_in=2)
    S.init(img)
    S.sweep(4)
    rho, ls, t = S.rho()
    rng = np.random.default_rng(5)
    pm = f32(np.log(rho.mean(axis=0)) + 0.05 * rng.standard_normal((H, W)))
    ps = f32(np.full((H, W), width) * np.exp(0.3 * rng.standard_normal((H, W))))
    S.set_block_proposal(pm, ps)
    S.set_block_beta(beta)
    O = oracle.OracleSampler(img.astype(np.float64), psf.astype(np.float64), g.astype(np.float64),
                             o.astype(np.float64), s.astype(np.float64), n_chains=C, seed=seed, burn_in=2)
    O.init()
    P = O.block_period()
    nbx = (W + 15) // 16
    n_dec = n_tie = 0
    worst = 0.0
    for k, colour in enumerate(colours):
        S.set_rho(rho, ls, t)
        dg, ag = S.block_colour(k + 3, colour)
        O.set_state(rho.astype(np.float64), ls.astype(np.float64), t)
        _, do, ao, sa = O.block_pass(k + 3, pm, ps, colour=colour, with_sabs=True, beta=beta)
        assert dg.shape == do.shape
        cy, cx = colour // P, colour % P
        nbx_c = (nbx - cx + P - 1) // P
        logu = np.empty_like(do)
        for c in range(C):
            for b in range(do.shape[1]):
                by, bx = cy + P * (b // nbx_c), cx + P * (b % nbx_c)
                logu[c, b] = math.log(oracle.uniform(seed, by * 16 * W + bx * 16, k + 3, c, 4))
        band = 1e-5 * (1.0 + sa)
        clear = np.abs(do - logu) > band
        err = np.abs(dg.astype(np.float64) - do) / (1.0 + sa)
        worst = max(worst, float(err.max()))
        bad = clear & (ag != ao)
        if bad.any() or err.max() >= 1e-5:
            say("  colour %d: worst err %.3g, mismatches %d; dg %s do %s logu %s" % (
                colour, err.max(), bad.sum(), dg[bad][:4], do[bad][:4], logu[bad][:4]))
        assert not bad.any()
        assert err.max() < 1e-5
        n_dec += do.size
        n_tie += int((~clear).sum())
        if clear.all():        # no tie: the committed blocks agree with the oracle's
            np.testing.assert_allclose(S.rho()[0], O.state()[0], rtol=3e-6)
    say("  %d block decisions, %d ties, max |dDelta|/(1+S) %.3g" % (n_dec, n_tie, worst))
    S.close()


def _lognormal_match(mean, var, widen):
    s2 = np.log1p(np.asarray(var) / np.asarray(mean) ** 2)
    return np.log(mean) - 0.5 * s2, widen * np.sqrt(s2)


def _block_only_draws(S, n_burn, n):
    S.block_move(n_burn)
    out = []
    for _ in range(n):
        S.block_move(1)
        out.append(S.rho()[0].copy())
    return np.array(out)


def _z(draws, exact_mean):
    """z-scores of the pooled mean with the standard error from the spread of
    the independent chains' means.  (Per-chain batch means would need batches
    longer than the rejection runs of a many-pixel independence move, which
    reach hundreds of passes.)"""
    n, C = draws.shape[:2]
    cm = draws.reshape(n, C, -1).mean(axis=0)
    se = cm.std(axis=0, ddof=1) / math.sqrt(C)
    return (cm.mean(axis=0) - np.ravel(exact_mean)) / se


def test_block_moves_alone_sample_the_identity_psf_posterior(bdc):
    from test_oracle_pins import one_pixel_posterior
    say("block moves alone: identity PSF closed form")
    rng = np.random.default_rng(23)
    H, W = 4, 4
    truth = rng.gamma(2.0, 15.0, (H, W)) + 1.0
    cam = synth.scmos_maps(rng, H, W)
    psf = np.array([[1.0]])
    img = f32(synth.simulate_frame(truth, psf, cam, rng))
    g, o, s = [f32(a) for a in cam.maps(H, W)]
    mv = np.array([[one_pixel_posterior(float(img[y, x]), float(g[y, x]), float(o[y, x]), float(s[y, x]))
                    for x in range(W)] for y in range(H)])
    pm, ps = _lognormal_match(mv[..., 0], mv[..., 1], 1.15)
    pm = pm + 0.03 * rng.standard_normal((H, W))
    S = bdc.Sampler(f32(psf), g, o, s, height=H, width=W, n_chains=64, seed=12)
    S.init(img)
    S.set_block_proposal(f32(pm), f32(ps))
    d = _block_only_draws(S, 200, 3000)
    acc, prop = S.block_stats()
    z = _z(d, mv[..., 0])
    say("  acceptance %.3f  max|z| %.2f mean z %.3f" % (acc / prop, np.abs(z).max(), z.mean()))
    assert np.all(np.abs(z) < 4.0)
    assert abs(z.mean()) < 1.2
    S.close()


@pytest.mark.parametrize("beta", [1.0, 0.4])
def test_block_moves_alone_match_two_pixel_quadrature(bdc, beta):
    from test_oracle_pins import two_pixel_posterior
    say("block moves alone: two-pixel quadrature, beta %.1f" % beta)
    w = np.array([140.0, 118.0])
    mean, var = two_pixel_posterior(w, 2.0, 100.0, 1.5)
    psf = np.zeros((3, 3), np.float32)
    psf[1] = [0.25, 0.5, 0.25]
    pm, ps = _lognormal_match(mean[None, :], var[None, :], 1.3)
    if beta < 1.0:
        pm = pm + 0.3
    S = bdc.Sampler(psf, np.float32(2.0), np.float32(100.0), np.float32(1.5), height=1, width=2,
                    n_chains=64, seed=13)
    S.init(f32(w[None, :]))
    S.set_block_proposal(f32(pm), f32(ps))
    S.set_block_beta(beta)
    d = _block_only_draws(S, 200, 3000)
    z = _z(d, mean)
    say("  z", z, "var", d.reshape(-1, 2).var(axis=0, ddof=1), var)
    assert np.all(np.abs(z) < 4.0)
    np.testing.assert_allclose(d.reshape(-1, 2).var(axis=0, ddof=1), var, rtol=0.08)
    S.close()


def test_init_learned_with_a_zero_network_is_its_definition(bdc):
    say("learned warm start, zero network")
    H, W = 37, 45
    img, psf, g, o, s, _ = _frame(H, W, synth.gaussian_psf(1.5, 11), seed=41)
    C, seed = 3, 19
    S = bdc.Sampler(psf, g, o, s, height=H, width=W, n_chains=C, seed=seed)
    S.init(img)
    net = bdc.UNet(4, 8, max_pixels=48 * 48)
    S.init_learned(net)
    rho, ls, t = S.rho()
    assert t == 0
    c = (img.astype(np.float64) - o) / g
    scale = c.mean()
    # m = s = 0: mean_log = log(scale), sd_log = 1, start spread min(2 sd_log, 3) = 2
    xi = np.array([[[oracle.normal(seed, y * W + x, 0, ch, 2) for x in range(W)] for y in range(H)]
                   for ch in range(C)])
    np.testing.assert_allclose(rho, scale * np.exp(2.0 * xi), rtol=4e-5)
    np.testing.assert_allclose(ls, -1.5)
    # block moves work from these maps and keep rho positive
    S.block_move(2)
    assert np.all(S.rho()[0] > 0)
    S.sweep(2)
    net.close()
    S.close()


# ---------------------------------------------------------------------------
# Block walk along what the blur removes (symmetric move in log rho)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("H,W,psf_kind,colours,step", [(70, 52, "gauss11", (0, 1, 3), 0.3),
                                                        (80, 96, "airy31", (0, 4, 8), 0.5),
                                                        (64, 64, "gauss11", (2,), 2.0)])
def test_block_walk_decisions_match_oracle(bdc, H, W, psf_kind, colours, step):
    say("block walk decisions %dx%d %s step %.2f" % (H, W, psf_kind, step))
    psf = synth.gaussian_psf(1.5, 11) if psf_kind == "gauss11" else synth.airy_psf(1.4, 0.6, 0.065, 31)
    img, psf, g, o, s, truth = _frame(H, W, psf, seed=37)
    C, seed = 2, 79
    S = bdc.Sampler(psf, g, o, s, height=H, width=W, n_chains=C, seed=seed, burn_in=2)
    S.init(img)
    S.sweep(4)
    rho, ls, t = S.rho()
    S.set_block_walk(step)
    O = oracle.OracleSampler(img.astype(np.float64), psf.astype(np.float64), g.astype(np.float64),
                             o.astype(np.float64), s.astype(np.float64), n_chains=C, seed=seed, burn_in=2)
    O.init()
    P = O.block_period()
    nbx = (W + 15) // 16
    n_dec = n_tie = n_acc = 0
    worst = 0.0
    for k, colour in enumerate(colours):
        S.set_rho(rho, ls, t)
        dg, ag = S.block_colour(k + 5, colour)
        O.set_state(rho.astype(np.float64), ls.astype(np.float64), t)
        _, do, ao, sa = O.block_pass(k + 5, 0.0, 1.0, colour=colour, with_sabs=True, walk=step)
        cy, cx = colour // P, colour % P
        nbx_c = (nbx - cx + P - 1) // P
        logu = np.empty_like(do)
        for c in range(C):
            for b in range(do.shape[1]):
                by, bx = cy + P * (b // nbx_c), cx + P * (b % nbx_c)
                logu[c, b] = math.log(oracle.uniform(seed, by * 16 * W + bx * 16, k + 5, c, 4))
        band = 1e-5 * (1.0 + sa)
        clear = np.abs(do - logu) > band
        err = np.abs(dg.astype(np.float64) - do) / (1.0 + sa)
        worst = max(worst, float(err.max()))
        bad = clear & (ag != ao)
        if bad.any() or err.max() >= 1e-5:
            say("  colour %d: worst err %.3g, mismatches %d" % (colour, err.max(), bad.sum()))
        assert not bad.any()
        assert err.max() < 1e-5
        n_dec += do.size
        n_tie += int((~clear).sum())
        n_acc += int(ao.sum())
        if clear.all():
            np.testing.assert_allclose(S.rho()[0], O.state()[0], rtol=3e-6)
    say("  %d block decisions (%d accepted), %d ties, max |dDelta|/(1+S) %.3g" % (n_dec, n_acc, n_tie, worst))
    S.close()


def test_block_walk_alone_matches_two_pixel_quadrature(bdc):
    from test_oracle_pins import two_pixel_posterior
    say("block walk alone: two-pixel quadrature")
    w = np.array([140.0, 118.0])
    mean, var = two_pixel_posterior(w, 2.0, 100.0, 1.5)
    psf = np.zeros((3, 3), np.float32)
    psf[1] = [0.25, 0.5, 0.25]
    S = bdc.Sampler(psf, np.float32(2.0), np.float32(100.0), np.float32(1.5), height=1, width=2,
                    n_chains=64, seed=17)
    S.init(f32(w[None, :]))
    S.set_block_walk(0.8)
    d = _block_only_draws(S, 300, 4000)
    acc, prop = S.block_stats()
    z = _z(d, mean)
    say("  acceptance %.3f  z %s" % (acc / prop, z))
    assert np.all(np.abs(z) < 4.0)
    np.testing.assert_allclose(d.reshape(-1, 2).var(axis=0, ddof=1), var, rtol=0.05)
    S.close()
