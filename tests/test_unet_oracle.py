"""Pins of the FP64 U-Net oracle (CPU): each layer against a library routine,
the whole backward pass against central finite differences, Adam against
torch's implementation.  None of them call the GPU library."""

import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import unet as U


def _rng(seed):
    return np.random.default_rng(seed)


def test_conv3_matches_library_cross_correlation():
    r = _rng(0)
    x = r.standard_normal((2, 7, 9, 5))
    W = r.standard_normal((4, 9, 5))
    b = r.standard_normal(4)
    y = U.conv3(x, W, b)
    wt = torch.from_numpy(W.reshape(4, 3, 3, 5).transpose(0, 3, 1, 2).copy())
    ref = F.conv2d(torch.from_numpy(x.transpose(0, 3, 1, 2).copy()), wt, torch.from_numpy(b), padding=1)
    np.testing.assert_allclose(y, ref.numpy().transpose(0, 2, 3, 1), rtol=1e-12, atol=1e-12)


def test_up2_matches_library_transposed_convolution():
    r = _rng(1)
    x = r.standard_normal((2, 3, 4, 6))
    W = r.standard_normal((4, 5, 6))          # [2*a + c][co][ci]
    b = r.standard_normal(5)
    y = U.up2(x, W, b)
    wt = torch.from_numpy(W.reshape(2, 2, 5, 6).transpose(3, 2, 0, 1).copy())   # [ci][co][a][c]
    ref = F.conv_transpose2d(torch.from_numpy(x.transpose(0, 3, 1, 2).copy()), wt, torch.from_numpy(b), stride=2)
    np.testing.assert_allclose(y, ref.numpy().transpose(0, 2, 3, 1), rtol=1e-12, atol=1e-12)


def test_maxpool_matches_library():
    r = _rng(2)
    x = r.standard_normal((2, 6, 8, 3))
    ref = F.max_pool2d(torch.from_numpy(x.transpose(0, 3, 1, 2).copy()), 2)
    np.testing.assert_array_equal(U.maxpool(x), ref.numpy().transpose(0, 2, 3, 1))


def test_layer_backward_passes_match_library_autograd():
    r = _rng(3)
    x = r.standard_normal((2, 6, 6, 4))
    W = r.standard_normal((3, 9, 4))
    gy = r.standard_normal((2, 6, 6, 3))
    gx, gW, gb = U.conv3_backward(x, W, gy)
    xt = torch.from_numpy(x.transpose(0, 3, 1, 2).copy()).requires_grad_()
    wt = torch.from_numpy(W.reshape(3, 3, 3, 4).transpose(0, 3, 1, 2).copy()).requires_grad_()
    bt = torch.zeros(3, dtype=torch.float64, requires_grad=True)
    F.conv2d(xt, wt, bt, padding=1).backward(torch.from_numpy(gy.transpose(0, 3, 1, 2).copy()))
    np.testing.assert_allclose(gx, xt.grad.numpy().transpose(0, 2, 3, 1), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(gW, wt.grad.numpy().transpose(0, 2, 3, 1).reshape(3, 9, 4), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(gb, bt.grad.numpy(), rtol=1e-11)

    x = r.standard_normal((2, 6, 6, 4))
    gy = r.standard_normal((2, 3, 3, 4))
    g = U.maxpool_backward(x, gy)
    xt = torch.from_numpy(x.transpose(0, 3, 1, 2).copy()).requires_grad_()
    F.max_pool2d(xt, 2).backward(torch.from_numpy(gy.transpose(0, 3, 1, 2).copy()))
    np.testing.assert_allclose(g, xt.grad.numpy().transpose(0, 2, 3, 1), rtol=1e-12)


def test_param_count_of_the_four_level_network():
    # 4 levels of 32/64/128/256 channels: about 1.93 M parameters
    n = U.param_count(4, 32)
    assert n == sum(co * 9 * ci + co if k == "conv" else (4 * co * ci + co if k == "up" else 2 * ci + 2)
                    for _, k, ci, co in U.layer_specs(4, 32))
    assert 1.90e6 < n < 1.96e6


@pytest.mark.parametrize("levels,base,hw", [(2, 8, 8), (3, 8, 8)])
def test_full_backward_matches_central_differences(levels, base, hw):
    r = _rng(10 + levels)
    p = U.init_params(levels, base, seed=levels)
    p += 0.05 * r.standard_normal(p.size)          # non-zero biases too
    x = np.abs(r.standard_normal((2, hw, hw))) + 0.2
    tgt = r.standard_normal((2, hw, hw, 2))
    loss, g = U.loss_and_grads(p, x, tgt, levels, base)
    idx = r.choice(p.size, 60, replace=False)
    # every layer's bias and weights get probed
    starts = np.cumsum([0] + [(co * 9 * ci if k == "conv" else (4 * co * ci if k == "up" else 2 * ci)) + co
                              for _, k, ci, co in U.layer_specs(levels, base)])
    idx = np.unique(np.concatenate([idx, starts[:-1], starts[1:] - 1]))
    eps = 1e-6
    num = []
    for i in idx:
        q = p.copy(); q[i] += eps
        lp = U.loss_and_grads(q, x, tgt, levels, base)[0]
        q[i] -= 2 * eps
        lm = U.loss_and_grads(q, x, tgt, levels, base)[0]
        num.append((lp - lm) / (2 * eps))
    num = np.array(num)
    np.testing.assert_allclose(g[idx], num, rtol=1e-4, atol=1e-7)


def test_adam_matches_library_optimiser():
    r = _rng(5)
    p0 = r.standard_normal(50)
    pt = torch.from_numpy(p0.copy()).requires_grad_()
    opt = torch.optim.Adam([pt], lr=1e-2)
    p, m1, m2 = p0.copy(), np.zeros(50), np.zeros(50)
    for step in range(1, 6):
        g = r.standard_normal(50)
        opt.zero_grad()
        pt.grad = torch.from_numpy(g.copy())
        opt.step()
        p, m1, m2 = U.adam_step(p, m1, m2, g, step, 1e-2)
    np.testing.assert_allclose(p, pt.detach().numpy(), rtol=1e-12, atol=1e-14)
