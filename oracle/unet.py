"""FP64 NumPy oracle of the learned warm-start network -- TEST INFRASTRUCTURE ONLY.

Only the test-suite may import this module.  It shares no code with the GPU
library.  It writes the network of ``include/bdc_unet.h`` out from its
definition, in float64, with plain NumPy slicing and einsum per 3x3 tap:

  * 3x3 convolution, zero padding:
        y[b, p, co] = bias[co] + sum_{tap, ci} W[co, tap, ci] x[b, p + off(tap), ci],
        off(tap) = (tap // 3 - 1, tap % 3 - 1)
  * ReLU after every 3x3 convolution;
  * 2x2 max pooling (stride 2);
  * 2x2 stride-2 transposed convolution:
        y[b, 2i + a, 2j + c, co] = bias[co] + sum_ci W[a, c, co, ci] x[b, i, j, ci]
  * skip concatenation: [up-sampled channels, skip channels];
  * 1x1 head with two outputs (m, s) per pixel;
  * loss  L = mean_p [(m_p - y_p)^2 + (s_p - z_p)^2];
  * Adam with bias correction.

The backward pass is reverse-mode differentiation of those definitions,
written out by hand; the tests pin it with central finite differences.
Parameter layout: as in bdc_unet.h (layers in forward order; 3x3 weights
[co][3][3][ci] then bias; transposed weights [2][2][co][ci] then bias; head
[2][c] then bias [2]).
"""

from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np


def layer_specs(levels: int, base: int) -> List[Tuple[str, str, int, int]]:
    """(name, kind, c_in, c_out) in forward order."""
    ch = [base << l for l in range(levels)]
    specs = []
    cin = 1
    for l in range(levels - 1):
        specs.append(("enc%d_1" % l, "conv", cin, ch[l]))
        specs.append(("enc%d_2" % l, "conv", ch[l], ch[l]))
        cin = ch[l]
    specs.append(("bott_1", "conv", ch[levels - 2], ch[levels - 1]))
    specs.append(("bott_2", "conv", ch[levels - 1], ch[levels - 1]))
    for l in range(levels - 2, -1, -1):
        specs.append(("up%d" % l, "up", ch[l + 1], ch[l]))
        specs.append(("dec%d_1" % l, "conv", 2 * ch[l], ch[l]))
        specs.append(("dec%d_2" % l, "conv", ch[l], ch[l]))
    specs.append(("head", "head", ch[0], 2))
    return specs


def param_count(levels: int, base: int) -> int:
    n = 0
    for _, kind, ci, co in layer_specs(levels, base):
        n += {"conv": co * 9 * ci, "up": 4 * co * ci, "head": 2 * ci}[kind] + co
    return n


def unpack(params: np.ndarray, levels: int, base: int) -> Dict[str, Tuple[np.ndarray, np.ndarray]]:
    """name -> (W, bias) views into the flat parameter vector."""
    out, k = {}, 0
    for name, kind, ci, co in layer_specs(levels, base):
        shape = {"conv": (co, 9, ci), "up": (4, co, ci), "head": (2, ci)}[kind]
        nw = int(np.prod(shape))
        out[name] = (params[k:k + nw].reshape(shape), params[k + nw:k + nw + co])
        k += nw + co
    return out


def init_params(levels: int, base: int, seed: int) -> np.ndarray:
    """He-normal weights and zero biases (a reproducible starting point)."""
    rng = np.random.default_rng(seed)
    parts = []
    for _, kind, ci, co in layer_specs(levels, base):
        fan_in = {"conv": 9 * ci, "up": ci, "head": ci}[kind]
        nw = {"conv": co * 9 * ci, "up": 4 * co * ci, "head": 2 * ci}[kind]
        std = np.sqrt(2.0 / fan_in) if kind != "head" else np.sqrt(1.0 / fan_in)
        parts.append(rng.standard_normal(nw) * std)
        parts.append(np.zeros(co))
    return np.concatenate(parts)


# --- layer definitions --------------------------------------------------------

def _offsets():
    return [(t // 3 - 1, t % 3 - 1) for t in range(9)]


def _shift(x, dy, dx):
    """xs[b, y, x] = x[b, y + dy, x + dx], zero outside."""
    B, H, W, C = x.shape
    out = np.zeros_like(x)
    ys, ye = max(0, -dy), min(H, H - dy)
    xs, xe = max(0, -dx), min(W, W - dx)
    out[:, ys:ye, xs:xe] = x[:, ys + dy:ye + dy, xs + dx:xe + dx]
    return out


def conv3(x, W, b):
    y = np.zeros(x.shape[:3] + (W.shape[0],))
    for t, (dy, dx) in enumerate(_offsets()):
        y += np.einsum("bhwc,oc->bhwo", _shift(x, dy, dx), W[:, t, :])
    return y + b


def conv3_backward(x, W, gy):
    """(gx, gW, gb) of y = conv3(x, W, b) for upstream gradient gy."""
    gW = np.zeros_like(W)
    gx = np.zeros_like(x)
    for t, (dy, dx) in enumerate(_offsets()):
        gW[:, t, :] = np.einsum("bhwo,bhwc->oc", gy, _shift(x, dy, dx))
        # x[p + off] feeds y[p]: the gradient flows back by the opposite shift
        gx += _shift(np.einsum("bhwo,oc->bhwc", gy, W[:, t, :]), -dy, -dx)
    return gx, gW, gy.sum(axis=(0, 1, 2))


def maxpool(x):
    B, H, W, C = x.shape
    v = x.reshape(B, H // 2, 2, W // 2, 2, C)
    return v.max(axis=(2, 4))


def maxpool_backward(x, gy):
    """Gradient to the first maximum of each 2x2 window (row-major order)."""
    B, H, W, C = x.shape
    win = x.reshape(B, H // 2, 2, W // 2, 2, C).transpose(0, 1, 3, 2, 4, 5).reshape(B, H // 2, W // 2, 4, C)
    arg = win.argmax(axis=3)
    g = np.zeros_like(win)
    np.put_along_axis(g, arg[:, :, :, None, :], gy[:, :, :, None, :], axis=3)
    return g.reshape(B, H // 2, W // 2, 2, 2, C).transpose(0, 1, 3, 2, 4, 5).reshape(B, H, W, C)


def up2(x, W, b):
    B, H, Wd, _ = x.shape
    co = W.shape[1]
    y = np.zeros((B, 2 * H, 2 * Wd, co))
    for a in range(2):
        for c in range(2):
            y[:, a::2, c::2, :] = np.einsum("bhwc,oc->bhwo", x, W[2 * a + c])
    return y + b


def up2_backward(x, W, gy):
    gx = np.zeros_like(x)
    gW = np.zeros_like(W)
    for a in range(2):
        for c in range(2):
            g = gy[:, a::2, c::2, :]
            gW[2 * a + c] = np.einsum("bhwo,bhwc->oc", g, x)
            gx += np.einsum("bhwo,oc->bhwc", g, W[2 * a + c])
    return gx, gW, gy.sum(axis=(0, 1, 2))


def relu(x):
    return np.maximum(x, 0.0)


# --- network ------------------------------------------------------------------

def forward(params, x, levels: int, base: int, keep: bool = False):
    """x: [B][H][W] -> out [B][H][W][2]; with keep, also the activations."""
    P = unpack(np.asarray(params, np.float64), levels, base)
    a = {"in0": np.asarray(x, np.float64)[..., None]}
    h = a["in0"]
    for l in range(levels - 1):
        a["ea%d" % l] = relu(conv3(h, *P["enc%d_1" % l]))
        a["skip%d" % l] = relu(conv3(a["ea%d" % l], *P["enc%d_2" % l]))
        h = a["in%d" % (l + 1)] = maxpool(a["skip%d" % l])
    a["ba"] = relu(conv3(h, *P["bott_1"]))
    src = a["bb"] = relu(conv3(a["ba"], *P["bott_2"]))
    for l in range(levels - 2, -1, -1):
        a["up%d" % l] = up2(src, *P["up%d" % l])
        a["cat%d" % l] = np.concatenate([a["up%d" % l], a["skip%d" % l]], axis=-1)
        a["da%d" % l] = relu(conv3(a["cat%d" % l], *P["dec%d_1" % l]))
        src = a["db%d" % l] = relu(conv3(a["da%d" % l], *P["dec%d_2" % l]))
    Wh, bh = P["head"]
    out = np.einsum("bhwc,oc->bhwo", src, Wh) + bh
    return (out, a) if keep else out


def loss_and_grads(params, x, target, levels: int, base: int):
    """(loss, flat gradient) of L = mean_p [(m - y)^2 + (s - z)^2]."""
    params = np.asarray(params, np.float64)
    P = unpack(params, levels, base)
    out, a = forward(params, x, levels, base, keep=True)
    target = np.asarray(target, np.float64)
    npx = out.shape[0] * out.shape[1] * out.shape[2]
    e = out - target
    loss = (e ** 2).sum() / npx
    grads = np.zeros_like(params)
    G = unpack(grads, levels, base)

    def put(name, gW, gb):
        G[name][0][...] = gW
        G[name][1][...] = gb

    gout = 2.0 * e / npx
    Wh, _ = P["head"]
    f = a["db0"]
    put("head", np.einsum("bhwo,bhwc->oc", gout, f), gout.sum(axis=(0, 1, 2)))
    g = np.einsum("bhwo,oc->bhwc", gout, Wh) * (f > 0)
    gskip = {}
    for l in range(levels - 1):
        gx, gW, gb = conv3_backward(a["da%d" % l], P["dec%d_2" % l][0], g)
        put("dec%d_2" % l, gW, gb)
        g = gx * (a["da%d" % l] > 0)
        gx, gW, gb = conv3_backward(a["cat%d" % l], P["dec%d_1" % l][0], g)
        put("dec%d_1" % l, gW, gb)
        c = a["up%d" % l].shape[-1]
        gup, gskip[l] = gx[..., :c], gx[..., c:]
        src = a["bb"] if l == levels - 2 else a["db%d" % (l + 1)]
        gx, gW, gb = up2_backward(src, P["up%d" % l][0], gup)
        put("up%d" % l, gW, gb)
        g = gx * (src > 0)
    gx, gW, gb = conv3_backward(a["ba"], P["bott_2"][0], g)
    put("bott_2", gW, gb)
    g = gx * (a["ba"] > 0)
    gx, gW, gb = conv3_backward(a["in%d" % (levels - 1)], P["bott_1"][0], g)
    put("bott_1", gW, gb)
    g = gx
    for l in range(levels - 2, -1, -1):
        g = (gskip[l] + maxpool_backward(a["skip%d" % l], g)) * (a["skip%d" % l] > 0)
        gx, gW, gb = conv3_backward(a["ea%d" % l], P["enc%d_2" % l][0], g)
        put("enc%d_2" % l, gW, gb)
        g = gx * (a["ea%d" % l] > 0)
        gx, gW, gb = conv3_backward(a["in%d" % l], P["enc%d_1" % l][0], g)
        put("enc%d_1" % l, gW, gb)
        g = gx
    return loss, grads


def adam_step(params, m1, m2, grads, step: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba) with bias correction; returns new (p, m1, m2)."""
    m1 = b1 * m1 + (1.0 - b1) * grads
    m2 = b2 * m2 + (1.0 - b2) * grads * grads
    mh = m1 / (1.0 - b1 ** step)
    vh = m2 / (1.0 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m1, m2
