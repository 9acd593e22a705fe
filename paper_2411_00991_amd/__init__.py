"""MI355X (gfx950) posterior sampler for physically motivated Bayesian deconvolution.

Python binding of the C ABI in ``include/bdc.h`` and ``include/bdc_unet.h`` (libbdc.so).  The functions
below carry the C names and only marshal arguments: numpy arrays are passed
as host pointers, CUDA/HIP torch tensors as device pointers on the current
torch stream.  Every step of the sampler runs in the HIP library; there is no
CPU fallback, and importing the binding fails if the library is missing.

Method: Hendrix et al., "Re-thinking Richardson-Lucy without Iteration
Cutoffs: Physically Motivated Bayesian Deconvolution" (arXiv:2411.00991),
Methods section (image formation, Eqs. 1-6; posterior, Eq. 9; parallelisation
by PSF-footprint locality).
"""

from __future__ import annotations

import ctypes
from typing import Optional, Tuple

import numpy as np

from . import _abi
from ._abi import (BDC_EDEVICE, BDC_EINVAL, BDC_ENOMEM, BDC_ENOTFINITE, BDC_ESTATE, BDC_OK,
                   BDC_PRIOR_FLAT, BDC_PRIOR_GAMMA, BDC_PRIOR_DIRICHLET, BDC_SCHED_AUTO, BDC_SCHED_BLOCK,
                   BDC_SCHED_BLOCK_SERIES, BDC_SCHED_BLOCK9_SERIES, BDC_SCHED_CHROMATIC, BDC_CAMERA_SCMOS,
                   BDC_CAMERA_EMCCD, bdc_config, bdc_unet_config)

_lib = _abi.load()

__all__ = ["BdcError", "bdc_config", "bdc_config_default", "bdc_create", "bdc_set_psf",
           "bdc_set_camera_maps", "bdc_init", "bdc_sweep", "bdc_posterior_moments", "bdc_rhat",
           "bdc_rhat_map", "bdc_window_mean", "bdc_mcse", "bdc_get_rho", "bdc_get_mu", "bdc_loglik",
           "bdc_logpost_trace", "bdc_accept_stats", "bdc_get_state", "bdc_set_state",
           "bdc_set_rho", "bdc_debug_run_groups", "bdc_schedule_info", "bdc_profile",
           "bdc_profile_read", "bdc_philox", "bdc_autotune", "bdc_set_schedule", "bdc_batch_create", "bdc_batch_sweep",
           "bdc_batch_check", "bdc_batch_info", "bdc_batch_last_error", "bdc_batch_destroy", "Batch",
           "bdc_last_error", "bdc_destroy", "Sampler",
           "bdc_unet_config", "bdc_unet_create", "bdc_unet_param_count", "bdc_unet_flops", "bdc_unet_set_params",
           "bdc_unet_get_params", "bdc_unet_forward", "bdc_unet_gradients", "bdc_unet_train_step",
           "bdc_unet_reset_optimizer", "bdc_unet_last_error", "bdc_unet_destroy", "bdc_init_learned",
           "bdc_set_block_proposal", "bdc_set_block_beta", "bdc_block_move", "bdc_block_stats", "bdc_debug_block_colour",
           "bdc_debug_gemm_bf16", "bdc_training_targets", "UNet"]


class BdcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (_abi.STATUS_NAMES.get(status, status), message))
        self.status = status


def _check(st: int, ctx) -> None:
    if st != BDC_OK:
        raise BdcError(st, bdc_last_error(ctx))


def _is_tensor(x) -> bool:
    return type(x).__module__.startswith("torch") and hasattr(x, "data_ptr")


def _arg(x, dtype):
    """(pointer, on_device, keep-alive) of an input array or tensor."""
    if x is None:
        return None, 0, None
    if _is_tensor(x):
        import torch
        tdt = {np.float32: torch.float32, np.uint32: torch.int32, np.uint8: torch.uint8}[dtype]
        if not x.is_contiguous() or (x.dtype != tdt and not (dtype is np.uint32 and x.dtype == torch.int32)):
            raise TypeError("tensor must be contiguous %s" % tdt)
        return ctypes.c_void_p(x.data_ptr()), int(x.is_cuda), x
    a = np.ascontiguousarray(x, dtype=dtype)
    return ctypes.c_void_p(a.ctypes.data), 0, a


def _stream_handle(stream) -> ctypes.c_void_p:
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        except Exception:
            pass
        return ctypes.c_void_p(None)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


# ---------------------------------------------------------------------------
# C-named entry points
# ---------------------------------------------------------------------------

def bdc_config_default(**overrides) -> bdc_config:
    cfg = bdc_config()
    _lib.bdc_config_default(ctypes.byref(cfg))
    for k, v in overrides.items():
        setattr(cfg, k, v)
    return cfg


def bdc_last_error(ctx=None) -> str:
    return _lib.bdc_last_error(ctx).decode()


def bdc_create(cfg: bdc_config, stream=None):
    out = ctypes.c_void_p()
    st = _lib.bdc_create(ctypes.byref(cfg), _stream_handle(stream), ctypes.byref(out))
    _check(st, None)
    return out


def bdc_destroy(ctx) -> None:
    _lib.bdc_destroy(ctx)


def bdc_set_psf(ctx, psf) -> None:
    p, dev, keep = _arg(psf, np.float32)
    shp = tuple(psf.shape)
    if len(shp) != 2:
        raise ValueError("psf must be 2-D")
    _check(_lib.bdc_set_psf(ctx, p, shp[0], shp[1], dev), ctx)


def bdc_set_camera_maps(ctx, gain, offset, sigma, per_pixel: Optional[bool] = None) -> None:
    if per_pixel is None:
        per_pixel = np.ndim(gain) == 2 if not _is_tensor(gain) else gain.dim() == 2
    args = [_arg(v, np.float32) for v in (gain, offset, sigma)]
    devs = {a[1] for a in args}
    if len(devs) != 1:
        raise ValueError("camera maps must all be host or all device")
    _check(_lib.bdc_set_camera_maps(ctx, args[0][0], args[1][0], args[2][0], int(per_pixel), devs.pop()), ctx)


def bdc_init(ctx, image, rho0=None) -> None:
    p, dev, k1 = _arg(image, np.float32)
    r, dev2, k2 = _arg(rho0, np.float32)
    if rho0 is not None and dev2 != dev:
        raise ValueError("image and rho0 must be on the same side")
    _check(_lib.bdc_init(ctx, p, r, dev), ctx)


def bdc_sweep(ctx, n: int) -> None:
    _check(_lib.bdc_sweep(ctx, int(n)), ctx)


def bdc_posterior_moments(ctx, mean, var, chain: int = -1) -> int:
    """Fills mean/var (either may be None); returns the per-chain sample count."""
    pm, dev, _ = _arg(mean, np.float32) if mean is not None else (None, None, None)
    pv, dev2, _ = _arg(var, np.float32) if var is not None else (None, None, None)
    dev = dev if dev is not None else (dev2 or 0)
    ns = ctypes.c_int64()
    _check(_lib.bdc_posterior_moments(ctx, chain, pm, pv, ctypes.byref(ns), dev), ctx)
    return ns.value


def bdc_diag_window(cfg: bdc_config, t: int):
    """(b_lo, half, b0, nb): the diagnostics' batch windows after t sweeps (host arithmetic)."""
    v = [ctypes.c_int32() for _ in range(4)]
    st = _lib.bdc_diag_window(ctypes.byref(cfg), ctypes.c_int64(t), *[ctypes.byref(x) for x in v])
    if st != BDC_OK:
        raise BdcError(st, "diag_window: no window after %d sweeps" % t)
    return tuple(x.value for x in v)


def bdc_richardson_lucy(ctx, n_iter: int, out) -> None:
    p, dev, _ = _arg(out, np.float32)
    _check(_lib.bdc_richardson_lucy(ctx, int(n_iter), p, dev), ctx)


def bdc_init_rl(ctx, n_iter: int) -> None:
    _check(_lib.bdc_init_rl(ctx, int(n_iter)), ctx)


def bdc_set_export(ctx, thin: int, capacity: int) -> None:
    _check(_lib.bdc_set_export(ctx, int(thin), int(capacity)), ctx)


def bdc_samples(ctx, out=None, first: int = 0, count: int = 0) -> int:
    """Stored samples [first, first + count) into out; returns the number stored."""
    ns = ctypes.c_int64()
    if out is None:
        _check(_lib.bdc_samples(ctx, None, 0, 0, ctypes.byref(ns), 0), ctx)
        return ns.value
    p, dev, _ = _arg(out, np.float32)
    _check(_lib.bdc_samples(ctx, p, int(first), int(count), ctypes.byref(ns), dev), ctx)
    return ns.value


def bdc_quantiles(ctx, probs, out) -> None:
    pr = np.ascontiguousarray(probs, np.float32)
    p, dev, _ = _arg(out, np.float32)
    _check(_lib.bdc_quantiles(ctx, ctypes.c_void_p(pr.ctypes.data), pr.size, p, dev), ctx)


def bdc_quantiles_of(samples, probs, out, stream=None) -> None:
    """Quantiles of device tensors: samples [n][n_pix], probs [n_probs] -> out [n_probs][n_pix]."""
    n, npix = samples.shape[0], int(np.prod(samples.shape[1:]))
    st = _lib.bdc_quantiles_of(ctypes.c_void_p(samples.data_ptr()), n, npix, ctypes.c_void_p(probs.data_ptr()),
                               probs.numel(), ctypes.c_void_p(out.data_ptr()), _stream_handle(stream))
    _check(st, None)


def bdc_cv_map(ctx, out) -> None:
    p, dev, _ = _arg(out, np.float32)
    _check(_lib.bdc_cv_map(ctx, p, dev), ctx)


def bdc_rhat(ctx) -> Tuple[float, float]:
    a, b = ctypes.c_float(), ctypes.c_float()
    _check(_lib.bdc_rhat(ctx, ctypes.byref(a), ctypes.byref(b)), ctx)
    return a.value, b.value


def bdc_rhat_map(ctx, out) -> None:
    p, dev, _ = _arg(out, np.float32)
    _check(_lib.bdc_rhat_map(ctx, p, dev), ctx)


def bdc_window_mean(ctx, out) -> None:
    p, dev, _ = _arg(out, np.float32)
    _check(_lib.bdc_window_mean(ctx, p, dev), ctx)


def bdc_mcse(ctx, out) -> None:
    p, dev, _ = _arg(out, np.float32)
    _check(_lib.bdc_mcse(ctx, p, dev), ctx)


def bdc_get_rho(ctx, rho, log_step=None) -> int:
    p1, dev, _ = _arg(rho, np.float32)
    p2, _, _ = _arg(log_step, np.float32)
    t = ctypes.c_int64()
    _check(_lib.bdc_get_rho(ctx, p1, p2, ctypes.byref(t), dev), ctx)
    return t.value


def bdc_get_mu(ctx, mu) -> None:
    p, dev, _ = _arg(mu, np.float32)
    _check(_lib.bdc_get_mu(ctx, p, dev), ctx)


def bdc_loglik(ctx, chain: int, ell) -> None:
    p, dev, _ = _arg(ell, np.float32)
    _check(_lib.bdc_loglik(ctx, chain, p, dev), ctx)


def bdc_logpost_trace(ctx, n_chains: int) -> np.ndarray:
    cnt = ctypes.c_int64()
    _check(_lib.bdc_logpost_trace(ctx, None, 0, ctypes.byref(cnt)), ctx)
    out = np.zeros((cnt.value, n_chains), np.float64)
    if cnt.value:
        _check(_lib.bdc_logpost_trace(ctx, ctypes.c_void_p(out.ctypes.data), cnt.value, ctypes.byref(cnt)), ctx)
    return out


def bdc_accept_stats(ctx, n_chains: int):
    a = np.zeros(n_chains, np.int64)
    p = np.zeros(n_chains, np.int64)
    _check(_lib.bdc_accept_stats(ctx, ctypes.c_void_p(a.ctypes.data), ctypes.c_void_p(p.ctypes.data)), ctx)
    return a, p


def bdc_get_state(ctx) -> bytes:
    n = ctypes.c_size_t()
    _check(_lib.bdc_get_state(ctx, None, ctypes.byref(n)), ctx)
    buf = (ctypes.c_char * n.value)()
    _check(_lib.bdc_get_state(ctx, buf, ctypes.byref(n)), ctx)
    return bytes(buf)


def bdc_set_state(ctx, state: bytes) -> None:
    buf = ctypes.create_string_buffer(state, len(state))
    _check(_lib.bdc_set_state(ctx, buf, len(state)), ctx)


def bdc_set_rho(ctx, rho, log_step, sweep: int) -> None:
    p1, dev, k1 = _arg(rho, np.float32)
    p2, dev2, k2 = _arg(log_step, np.float32)
    if dev != dev2:
        raise ValueError("rho and log_step must be on the same side")
    _check(_lib.bdc_set_rho(ctx, p1, p2, int(sweep), dev), ctx)


def bdc_debug_run_groups(ctx, g0: int, g1: int, delta, accepted) -> None:
    p1, dev, _ = _arg(delta, np.float32)
    p2, _, _ = _arg(accepted, np.uint8)
    _check(_lib.bdc_debug_run_groups(ctx, g0, g1, p1, p2, dev), ctx)


def bdc_schedule_info(ctx):
    n, s, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.bdc_schedule_info(ctx, ctypes.byref(n), ctypes.byref(s), ctypes.byref(b)), ctx)
    return n.value, s.value, b.value


def bdc_profile(ctx, enable: bool) -> None:
    _check(_lib.bdc_profile(ctx, int(bool(enable))), ctx)


def bdc_profile_read(ctx):
    """Returns (ms[3], launches[3], work[6]) since the last read (see bdc.h)."""
    ms = np.zeros(3, np.float64)
    ln = np.zeros(3, np.int64)
    wk = np.zeros(6, np.int64)
    _check(_lib.bdc_profile_read(ctx, ctypes.c_void_p(ms.ctypes.data), ctypes.c_void_p(ln.ctypes.data),
                                 ctypes.c_void_p(wk.ctypes.data)), ctx)
    return ms, ln, wk


def bdc_autotune(ctx, blocks, sweeps: int):
    """Times each candidate block side (0 = chromatic scan); returns (ms per sweep, best)."""
    b = np.ascontiguousarray(blocks, np.int32)
    ms = np.zeros(b.size, np.float32)
    best = ctypes.c_int32()
    _check(_lib.bdc_autotune(ctx, ctypes.c_void_p(b.ctypes.data), b.size, int(sweeps),
                             ctypes.c_void_p(ms.ctypes.data), ctypes.byref(best)), ctx)
    return ms, best.value


def bdc_set_schedule(ctx, schedule: int, block: int = 0) -> None:
    _check(_lib.bdc_set_schedule(ctx, int(schedule), int(block)), ctx)


def bdc_batch_last_error(batch=None) -> str:
    return _lib.bdc_batch_last_error(batch).decode()


def _bcheck(st: int, batch) -> None:
    if st != BDC_OK:
        raise BdcError(st, bdc_batch_last_error(batch))


def bdc_batch_create(ctxs, stream=None):
    arr = (ctypes.c_void_p * len(ctxs))(*[c.value for c in ctxs])
    out = ctypes.c_void_p()
    _bcheck(_lib.bdc_batch_create(arr, len(ctxs), _stream_handle(stream), ctypes.byref(out)), None)
    return out


def bdc_batch_sweep(batch, n: int) -> None:
    _bcheck(_lib.bdc_batch_sweep(batch, int(n)), batch)


def bdc_batch_check(batch) -> None:
    _bcheck(_lib.bdc_batch_check(batch), batch)


def bdc_batch_info(batch):
    n, g, l = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
    _bcheck(_lib.bdc_batch_info(batch, ctypes.byref(n), ctypes.byref(g), ctypes.byref(l)), batch)
    return n.value, g.value, l.value


def bdc_batch_destroy(batch) -> None:
    _lib.bdc_batch_destroy(batch)


def bdc_philox(ctr, key0: int, key1: int, out, stream=None) -> None:
    """Device Philox4x32-10 of [n, 4] counters (int32/uint32 CUDA tensors)."""
    n = ctr.shape[0]
    _check(_lib.bdc_philox(ctypes.c_void_p(ctr.data_ptr()), n, key0 & 0xFFFFFFFF, key1 & 0xFFFFFFFF,
                           ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)), None)


# ---------------------------------------------------------------------------
# Convenience object over one context (device buffers from torch)
# ---------------------------------------------------------------------------

class Sampler:
    """One frame's posterior sampler.  Inputs may be numpy arrays or tensors."""

    def __init__(self, psf, gain, offset, sigma, *, height: int, width: int, n_chains: int = 1,
                 seed: int = 0, burn_in: int = 0, log_step0: float = -1.5,
                 schedule: int = BDC_SCHED_AUTO, block_size: int = 0,
                 prior_kind: int = BDC_PRIOR_FLAT, prior_a: float = 1.0, prior_b: float = 0.0,
                 rhat_block: int = 25, max_sweeps: int = 4096, camera: int = BDC_CAMERA_SCMOS,
                 object_sub: int = 1, stream=None):
        """height x width is the camera frame; with object_sub = k > 1 the object
        (state, draws, moments and their maps) lives on a (k height) x (k width)
        lattice and the PSF is sampled on it."""
        self.cfg = bdc_config_default(height=height, width=width, n_chains=n_chains, seed=seed,
                                      burn_in=burn_in, log_step0=log_step0, schedule=schedule,
                                      block_size=block_size, prior_kind=prior_kind, prior_a=prior_a,
                                      prior_b=prior_b, rhat_block=rhat_block, max_sweeps=max_sweeps,
                                      camera=camera, object_sub=object_sub)
        k = max(1, object_sub)
        self.H, self.W, self.C = height, width, n_chains
        self.Ho, self.Wo = k * height, k * width
        self.ctx = bdc_create(self.cfg, stream)
        try:
            bdc_set_psf(self.ctx, psf)
            bdc_set_camera_maps(self.ctx, gain, offset, sigma)
        except Exception:
            self.close()
            raise

    def close(self) -> None:
        if getattr(self, "ctx", None) is not None and _lib is not None:
            bdc_destroy(self.ctx)
        self.ctx = None

    def __del__(self):
        self.close()

    def init(self, image, rho0=None) -> None:
        bdc_init(self.ctx, image, rho0)

    def sweep(self, n: int) -> None:
        bdc_sweep(self.ctx, n)

    def moments(self, chain: int = -1):
        mean = np.empty((self.Ho, self.Wo), np.float32)
        var = np.empty((self.Ho, self.Wo), np.float32)
        n = bdc_posterior_moments(self.ctx, mean, var, chain)
        return mean, var, n

    def rho(self):
        rho = np.empty((self.C, self.Ho, self.Wo), np.float32)
        ls = np.empty((self.C, self.Ho, self.Wo), np.float32)
        t = bdc_get_rho(self.ctx, rho, ls)
        return rho, ls, t

    def mu(self):
        mu = np.empty((self.C, self.H, self.W), np.float32)
        bdc_get_mu(self.ctx, mu)
        return mu

    def loglik(self, chain: int = 0):
        ell = np.empty((self.H, self.W), np.float32)
        bdc_loglik(self.ctx, chain, ell)
        return ell

    def rhat(self):
        return bdc_rhat(self.ctx)

    def rhat_map(self):
        out = np.empty((self.Ho, self.Wo), np.float32)
        bdc_rhat_map(self.ctx, out)
        return out

    def mcse(self):
        out = np.empty((self.Ho, self.Wo), np.float32)
        bdc_mcse(self.ctx, out)
        return out

    def window_mean(self):
        out = np.empty((self.Ho, self.Wo), np.float32)
        bdc_window_mean(self.ctx, out)
        return out

    def accept_stats(self):
        return bdc_accept_stats(self.ctx, self.C)

    def richardson_lucy(self, n_iter: int):
        out = np.empty((self.Ho, self.Wo), np.float32)
        bdc_richardson_lucy(self.ctx, n_iter, out)
        return out

    def init_rl(self, n_iter: int) -> None:
        bdc_init_rl(self.ctx, n_iter)

    def set_export(self, thin: int, capacity: int) -> None:
        bdc_set_export(self.ctx, thin, capacity)

    def samples(self, first: int = 0, count: Optional[int] = None):
        n = bdc_samples(self.ctx)
        count = n - first if count is None else count
        out = np.empty((count, self.C, self.Ho, self.Wo), np.float32)
        if count:
            bdc_samples(self.ctx, out, first, count)
        return out

    def quantiles(self, probs):
        out = np.empty((len(probs), self.Ho, self.Wo), np.float32)
        bdc_quantiles(self.ctx, probs, out)
        return out

    def cv_map(self):
        out = np.empty((self.Ho, self.Wo), np.float32)
        bdc_cv_map(self.ctx, out)
        return out

    def trace(self):
        return bdc_logpost_trace(self.ctx, self.C)

    def set_rho(self, rho, log_step, sweep: int) -> None:
        bdc_set_rho(self.ctx, np.asarray(rho, np.float32), np.asarray(log_step, np.float32), sweep)

    def run_groups(self, g0: int, g1: int):
        delta = np.empty((self.C, self.Ho, self.Wo), np.float32)
        acc = np.empty((self.C, self.Ho, self.Wo), np.uint8)
        bdc_debug_run_groups(self.ctx, g0, g1, delta, acc)
        return delta, acc

    def schedule_info(self):
        return bdc_schedule_info(self.ctx)

    def profile(self, enable: bool = True) -> None:
        bdc_profile(self.ctx, enable)

    def profile_read(self):
        return bdc_profile_read(self.ctx)

    def autotune(self, blocks, sweeps: int = 2):
        return bdc_autotune(self.ctx, blocks, sweeps)

    def set_schedule(self, schedule: int, block: int = 0) -> None:
        bdc_set_schedule(self.ctx, schedule, block)

    def get_state(self) -> bytes:
        return bdc_get_state(self.ctx)

    def set_state(self, state: bytes) -> None:
        bdc_set_state(self.ctx, state)

    def init_learned(self, net: "UNet") -> None:
        bdc_init_learned(self.ctx, net.handle)

    def set_block_proposal(self, mean_log, sd_log) -> None:
        bdc_set_block_proposal(self.ctx, mean_log, sd_log)

    def block_move(self, n: int = 1) -> None:
        bdc_block_move(self.ctx, n)

    def set_block_beta(self, beta: float) -> None:
        bdc_set_block_beta(self.ctx, beta)

    def set_block_walk(self, step: float) -> None:
        bdc_set_block_walk(self.ctx, step)

    def block_stats(self):
        return bdc_block_stats(self.ctx)

    def training_targets(self, x=None, target=None):
        """(x [H][W], target [H][W][2], scale); device tensors are filled in place."""
        if x is None:
            x = np.empty((self.Ho, self.Wo), np.float32)
            target = np.empty((self.Ho, self.Wo, 2), np.float32)
        sc = bdc_training_targets(self.ctx, x, target)
        return x, target, sc

    def block_colour(self, pass_index: int, colour: int):
        return bdc_debug_block_colour(self.ctx, pass_index, colour, self.C, self.H * self.W)


class Batch:
    """Several initialised Samplers advanced together by one graph launch per sweep."""

    def __init__(self, samplers, stream=None):
        self.samplers = list(samplers)
        self.handle = bdc_batch_create([sp.ctx for sp in self.samplers], stream)

    def sweep(self, n: int) -> None:
        bdc_batch_sweep(self.handle, n)

    def check(self) -> None:
        bdc_batch_check(self.handle)

    def info(self):
        return bdc_batch_info(self.handle)

    def close(self) -> None:
        if getattr(self, "handle", None) is not None and _lib is not None:
            bdc_batch_destroy(self.handle)
        self.handle = None

    def __del__(self):
        self.close()


# ---------------------------------------------------------------------------
# The learned part (include/bdc_unet.h)
# ---------------------------------------------------------------------------

def bdc_unet_last_error(u=None) -> str:
    return _lib.bdc_unet_last_error(u).decode()


def _ucheck(st: int, u) -> None:
    if st != BDC_OK:
        raise BdcError(st, bdc_unet_last_error(u))


def bdc_unet_create(levels: int, base_channels: int, max_pixels: int, training: bool, stream=None):
    cfg = bdc_unet_config(levels=levels, base_channels=base_channels, max_pixels=max_pixels,
                          training=int(bool(training)))
    out = ctypes.c_void_p()
    _ucheck(_lib.bdc_unet_create(ctypes.byref(cfg), _stream_handle(stream), ctypes.byref(out)), None)
    return out


def bdc_unet_destroy(u) -> None:
    _lib.bdc_unet_destroy(u)


def bdc_unet_param_count(u) -> int:
    n = ctypes.c_int64()
    _ucheck(_lib.bdc_unet_param_count(u, ctypes.byref(n)), u)
    return n.value


def bdc_unet_flops(u, batch: int, height: int, width: int) -> float:
    f = ctypes.c_double()
    _ucheck(_lib.bdc_unet_flops(u, batch, height, width, ctypes.byref(f)), u)
    return f.value


def bdc_unet_set_params(u, params) -> None:
    p, dev, _ = _arg(params, np.float32)
    _ucheck(_lib.bdc_unet_set_params(u, p, dev), u)


def bdc_unet_get_params(u, params) -> None:
    p, dev, _ = _arg(params, np.float32)
    _ucheck(_lib.bdc_unet_get_params(u, p, dev), u)


def _shape3(x):
    shp = tuple(x.shape)
    if len(shp) != 3:
        raise ValueError("x must be [batch][height][width]")
    return shp


def bdc_unet_forward(u, x, out) -> None:
    b, h, w = _shape3(x)
    px, dev, _ = _arg(x, np.float32)
    po, dev2, _ = _arg(out, np.float32)
    if dev != dev2:
        raise ValueError("x and out must be on the same side")
    _ucheck(_lib.bdc_unet_forward(u, px, b, h, w, po, dev), u)


def bdc_unet_gradients(u, x, target, grads=None) -> float:
    b, h, w = _shape3(x)
    px, dev, _ = _arg(x, np.float32)
    pt, dev2, _ = _arg(target, np.float32)
    pg, dev3, _ = _arg(grads, np.float32)
    if dev != dev2 or (grads is not None and dev3 != dev):
        raise ValueError("x, target and grads must be on the same side")
    loss = ctypes.c_float()
    _ucheck(_lib.bdc_unet_gradients(u, px, pt, b, h, w, pg, ctypes.byref(loss), dev), u)
    return loss.value


def bdc_unet_train_step(u, x, target, lr: float, want_loss: bool = True):
    b, h, w = _shape3(x)
    px, dev, _ = _arg(x, np.float32)
    pt, dev2, _ = _arg(target, np.float32)
    if dev != dev2:
        raise ValueError("x and target must be on the same side")
    loss = ctypes.c_float()
    _ucheck(_lib.bdc_unet_train_step(u, px, pt, b, h, w, float(lr), ctypes.byref(loss) if want_loss else None,
                                     dev), u)
    return loss.value if want_loss else None


def bdc_debug_gemm_bf16(a_bits: np.ndarray, b_bits: np.ndarray) -> np.ndarray:
    """C = A B^T on the matrix cores; A [M][K], B [N][K] as uint16 BF16 patterns."""
    a = np.ascontiguousarray(a_bits, np.uint16)
    b = np.ascontiguousarray(b_bits, np.uint16)
    m, k = a.shape
    n = b.shape[0]
    c = np.empty((m, n), np.float32)
    _ucheck(_lib.bdc_debug_gemm_bf16(ctypes.c_void_p(a.ctypes.data), ctypes.c_void_p(b.ctypes.data),
                                     ctypes.c_void_p(c.ctypes.data), m, n, k), None)
    return c


def bdc_unet_reset_optimizer(u) -> None:
    _ucheck(_lib.bdc_unet_reset_optimizer(u), u)


def bdc_init_learned(ctx, u) -> None:
    _check(_lib.bdc_init_learned(ctx, u), ctx)


def bdc_set_block_proposal(ctx, mean_log, sd_log) -> None:
    p1, dev, _k1 = _arg(mean_log, np.float32)
    p2, dev2, _k2 = _arg(sd_log, np.float32)
    if dev != dev2:
        raise ValueError("mean_log and sd_log must be on the same side")
    _check(_lib.bdc_set_block_proposal(ctx, p1, p2, dev), ctx)


def bdc_set_block_beta(ctx, beta: float) -> None:
    _check(_lib.bdc_set_block_beta(ctx, float(beta)), ctx)


def bdc_set_block_walk(ctx, step: float) -> None:
    _check(_lib.bdc_set_block_walk(ctx, ctypes.c_float(step)), ctx)


def bdc_block_move(ctx, n: int) -> None:
    _check(_lib.bdc_block_move(ctx, int(n)), ctx)


def bdc_block_stats(ctx):
    a, p = ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.bdc_block_stats(ctx, ctypes.byref(a), ctypes.byref(p)), ctx)
    return a.value, p.value


def bdc_training_targets(ctx, x, target) -> float:
    """Fills the network input x [H][W] and target [H][W][2]; returns the frame scale."""
    px, dev, _ = _arg(x, np.float32)
    pt, dev2, _ = _arg(target, np.float32)
    if dev != dev2:
        raise ValueError("x and target must be on the same side")
    sc = ctypes.c_float()
    _check(_lib.bdc_training_targets(ctx, px, pt, ctypes.byref(sc), dev), ctx)
    return sc.value


def bdc_training_targets_noalloc(ctx, x, target) -> float:
    """bdc_training_targets without device allocation (library scratch staging)."""
    px, dev, _ = _arg(x, np.float32)
    pt, dev2, _ = _arg(target, np.float32)
    if dev != dev2:
        raise ValueError("x and target must be on the same side")
    sc = ctypes.c_float()
    _check(_lib.bdc_training_targets_noalloc(ctx, px, pt, ctypes.byref(sc), dev), ctx)
    return sc.value


def bdc_debug_block_colour(ctx, pass_index: int, colour: int, n_chains: int, max_blocks: int):
    """(delta [chains][blocks], accepted [chains][blocks]) of one block colour."""
    delta = np.zeros(n_chains * max_blocks, np.float32)
    acc = np.zeros(n_chains * max_blocks, np.uint8)
    nb = ctypes.c_int32()
    _check(_lib.bdc_debug_block_colour(ctx, int(pass_index), int(colour), ctypes.c_void_p(delta.ctypes.data),
                                       ctypes.c_void_p(acc.ctypes.data), ctypes.byref(nb)), ctx)
    n = nb.value
    return delta[:n_chains * n].reshape(n_chains, n), acc[:n_chains * n].reshape(n_chains, n)


class UNet:
    """The learned warm-start / block-proposal network (BF16 MFMA kernels)."""

    def __init__(self, levels: int = 4, base_channels: int = 32, max_pixels: int = 1 << 20,
                 training: bool = False, stream=None):
        self.levels, self.base = levels, base_channels
        self.handle = bdc_unet_create(levels, base_channels, max_pixels, training, stream)
        self.n_params = bdc_unet_param_count(self.handle)

    def close(self) -> None:
        if getattr(self, "handle", None) is not None and _lib is not None:
            bdc_unet_destroy(self.handle)
        self.handle = None

    def __del__(self):
        self.close()

    def set_params(self, params) -> None:
        bdc_unet_set_params(self.handle, params)

    def get_params(self) -> np.ndarray:
        out = np.empty(self.n_params, np.float32)
        bdc_unet_get_params(self.handle, out)
        return out

    def forward(self, x):
        """x: [B][H][W] float32 (numpy or device tensor) -> [B][H][W][2] on the same side."""
        if _is_tensor(x):
            import torch
            out = torch.empty(tuple(x.shape) + (2,), dtype=torch.float32, device=x.device)
        else:
            x = np.ascontiguousarray(x, np.float32)
            out = np.empty(x.shape + (2,), np.float32)
        bdc_unet_forward(self.handle, x, out)
        return out

    def gradients(self, x, target):
        """(loss, FP32 gradients in the parameter layout) without an update."""
        grads = np.empty(self.n_params, np.float32)
        if _is_tensor(x):
            import torch
            g = torch.empty(self.n_params, dtype=torch.float32, device=x.device)
            loss = bdc_unet_gradients(self.handle, x, target, g)
            torch.cuda.synchronize()
            return loss, g.cpu().numpy()
        loss = bdc_unet_gradients(self.handle, np.ascontiguousarray(x, np.float32),
                                  np.ascontiguousarray(target, np.float32), grads)
        return loss, grads

    def train_step(self, x, target, lr: float, want_loss: bool = True):
        return bdc_unet_train_step(self.handle, x, target, lr, want_loss)

    def flops(self, batch: int, height: int, width: int) -> float:
        return bdc_unet_flops(self.handle, batch, height, width)

    def reset_optimizer(self) -> None:
        bdc_unet_reset_optimizer(self.handle)
