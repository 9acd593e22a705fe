"""The learned warm start and block proposal, end to end.

1. Training data: the batched sampler runs on many synthetic frames; each
   frame's pooled posterior moments become a (network input, target) pair on
   the device (``bdc_training_targets``).
2. Training: the U-Net's own forward/backward/Adam kernels
   (``bdc_unet_train_step``) on random mini-batches with random flips.
3. Use: ``bdc_init_learned`` (network inference, per-pixel log-normal maps,
   chains started from them) and ``bdc_block_move`` interleaved with sweeps.
4. Compare: wall time and sweeps until the convergence criterion (99th
   percentile of the per-pixel split-R-hat and the R-hat of the log-posterior
   trace both below 1.01), and the posterior-mean error at that point,
   plain start against learned start.

All computation runs in libbdc.so; torch provides device memory only.
"""

from __future__ import annotations

import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import Batch, Sampler, UNet


def layer_shapes(levels: int, base: int):
    """(kind, c_in, c_out) of every layer in the parameter order of bdc_unet.h."""
    ch = [base << l for l in range(levels)]
    out, cin = [], 1
    for l in range(levels - 1):
        out += [("conv", cin, ch[l]), ("conv", ch[l], ch[l])]
        cin = ch[l]
    out += [("conv", ch[levels - 2], ch[levels - 1]), ("conv", ch[levels - 1], ch[levels - 1])]
    for l in range(levels - 2, -1, -1):
        out += [("up", ch[l + 1], ch[l]), ("conv", 2 * ch[l], ch[l]), ("conv", ch[l], ch[l])]
    out.append(("head", ch[0], 2))
    return out


def param_count(levels: int, base: int) -> int:
    n = 0
    for kind, ci, co in layer_shapes(levels, base):
        n += {"conv": co * 9 * ci, "up": 4 * co * ci, "head": 2 * ci}[kind] + co
    return n


def he_init(levels: int, base: int, seed: int, head_bias=(0.0, -1.5)) -> np.ndarray:
    """He-normal weights, zero biases; the head's log-std bias starts at
    head_bias[1] (a proposal width of exp(-1.5) ~ 0.22 in log rho)."""
    rng = np.random.default_rng(seed)
    parts = []
    for kind, ci, co in layer_shapes(levels, base):
        if kind == "conv":
            parts += [rng.standard_normal(co * 9 * ci) * np.sqrt(2.0 / (9 * ci)), np.zeros(co)]
        elif kind == "up":
            parts += [rng.standard_normal(4 * co * ci) * np.sqrt(2.0 / ci), np.zeros(co)]
        else:
            parts += [rng.standard_normal(2 * ci) * np.sqrt(1.0 / ci) * 0.1, np.asarray(head_bias, np.float64)]
    return np.concatenate(parts).astype(np.float32)


def _cam(fr):
    H, W = fr.image.shape
    return [np.asarray(a, np.float32) for a in fr.camera.maps(H, W)]


def make_sampler(fr, n_chains: int, seed: int, burn_in: int, max_sweeps: int, rhat_block: int = 25,
                 schedule: int = 0, prior_kind: int = 0) -> Sampler:
    H, W = fr.image.shape
    g, o, s = _cam(fr)
    sp = Sampler(np.asarray(fr.psf, np.float32), g, o, s, height=H, width=W, n_chains=n_chains, seed=seed,
                 burn_in=burn_in, max_sweeps=max_sweeps, rhat_block=rhat_block, schedule=schedule,
                 prior_kind=prior_kind)
    sp.init(np.asarray(fr.image, np.float32))
    return sp


def generate(frames: Sequence, sweeps: int, burn_in: int, chains: int = 1, log=None):
    """Training pairs of equally sized frames: (X [n][H][W], T [n][H][W][2]) as
    device tensors, from `sweeps` batched sweeps per frame."""
    import torch
    H, W = frames[0].image.shape
    samplers = [make_sampler(fr, chains, fr.seed, burn_in, sweeps + 4) for fr in frames]
    batch = Batch(samplers)
    t0 = time.perf_counter()
    done = 0
    while done < sweeps:
        k = min(50, sweeps - done)
        batch.sweep(k)
        batch.check()
        done += k
        if log:
            log("  data: %d/%d sweeps over %d frames" % (done, sweeps, len(frames)))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    X = torch.empty((len(frames), H, W), dtype=torch.float32, device="cuda")
    T = torch.empty((len(frames), H, W, 2), dtype=torch.float32, device="cuda")
    for i, sp in enumerate(samplers):
        sp.training_targets(X[i], T[i])
    torch.cuda.synchronize()
    batch.close()
    for sp in samplers:
        sp.close()
    updates = float(len(frames) * H * W * chains * sweeps)
    return X, T, {"seconds": el, "pixel_updates": updates}


def train(net: UNet, X, T, steps: int, batch: int, lr: float, seed: int = 0, log=None,
          log_every: int = 100) -> List[float]:
    """Adam on random mini-batches with random horizontal/vertical flips."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    n = X.shape[0]
    losses = []
    for it in range(steps):
        idx = torch.randint(0, n, (batch,), generator=g).to(X.device)
        xb, tb = X.index_select(0, idx), T.index_select(0, idx)
        if torch.rand(1, generator=g).item() < 0.5:
            xb, tb = xb.flip(1), tb.flip(1)
        if torch.rand(1, generator=g).item() < 0.5:
            xb, tb = xb.flip(2), tb.flip(2)
        want = (it % log_every == 0) or it == steps - 1
        loss = net.train_step(xb.contiguous(), tb.contiguous(), lr, want_loss=want)
        if want:
            losses.append(loss)
            if log:
                log("  train step %d loss %.4f" % (it, loss))
    return losses


def run_to_rhat(sp: Sampler, max_sweeps: int, check_every: int = 25, block_every: int = 0,
                threshold: float = 1.01, truth_mean: Optional[np.ndarray] = None, log=None) -> Dict:
    """Sweeps (with a block move after every `block_every`-th sweep when > 0) until
    the 99th percentile of the split-R-hat map and the log-posterior R-hat are
    both below `threshold`, checked every `check_every` sweeps.  Returns the
    sweep count, wall seconds (from the call, checks included) and the history."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = []
    done = 0
    converged = False
    while done < max_sweeps:
        if block_every > 0:
            for _ in range(check_every):
                sp.sweep(1)
                done += 1
                if done % block_every == 0:
                    sp.block_move(1)
        else:
            sp.sweep(check_every)
            done += check_every
        if done >= 4 * sp.cfg.rhat_block:
            p99, rlp = sp.rhat()
            hist.append((done, time.perf_counter() - t0, float(p99), float(rlp)))
            if log:
                log("  sweep %d: R-hat p99 %.4f, log-posterior %.4f" % (done, p99, rlp))
            if p99 < threshold and rlp < threshold:
                converged = True
                break
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out = {"sweeps": done, "seconds": el, "converged": converged, "history": hist}
    if truth_mean is not None and hist:
        mean = sp.window_mean()
        out["rmse"] = float(np.sqrt(np.mean((mean - truth_mean) ** 2)))
    return out
