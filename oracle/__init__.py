"""FP64 CPU oracle of the posterior sampler -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It wraps ``oracle.c`` (plain C, double precision), which
shares no code with the GPU library; see that file's header for what it
computes and which passages of the paper each part follows.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, ENOMEM = 0, -1, -2
SCHED_CHROMATIC, SCHED_BLOCK, SCHED_BLOCK9 = 1, 2, 3
PRIOR_FLAT, PRIOR_GAMMA, PRIOR_DIRICHLET = 0, 1, 2
CAMERA_SCMOS, CAMERA_EMCCD = 0, 1


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (FP64, OpenMP across same-group pixels)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class OrcConfig(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("s", ctypes.c_int32),
                ("n_chains", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("block", ctypes.c_int32), ("prior_kind", ctypes.c_int32),
                ("burn_in", ctypes.c_int32), ("prior_a", ctypes.c_double),
                ("prior_b", ctypes.c_double), ("log_step0", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("camera", ctypes.c_int32), ("sub", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.orc_philox_many.argtypes = [u32p, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint32, u32p]
        L.orc_normal.restype = ctypes.c_double
        L.orc_normal.argtypes = [ctypes.c_uint64] + [ctypes.c_uint32] * 4
        L.orc_uniform.restype = ctypes.c_double
        L.orc_uniform.argtypes = [ctypes.c_uint64] + [ctypes.c_uint32] * 4
        L.orc_loglik_pixel.restype = ctypes.c_double
        L.orc_loglik_pixel.argtypes = [ctypes.c_double] * 5
        L.orc_loglik_many.argtypes = [dp] * 5 + [ctypes.c_int64, dp]
        L.orc_loglik_emccd_many.argtypes = [dp] * 5 + [ctypes.c_int64, dp]
        L.orc_forward.argtypes = [dp, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, dp]
        L.orc_forward_sub.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, dp]
        L.orc_create.argtypes = [ctypes.POINTER(OrcConfig), dp, dp, dp, dp, dp,
                                 ctypes.POINTER(ctypes.c_void_p)]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_init.argtypes = [ctypes.c_void_p, dp]
        L.orc_log_posterior.restype = ctypes.c_double
        L.orc_log_posterior.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_sweeps.argtypes = [ctypes.c_void_p, ctypes.c_int, dp]
        L.orc_run_groups.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, dp, dp, ctypes.POINTER(ctypes.c_uint8), dp]
        L.orc_set_state.argtypes = [ctypes.c_void_p, dp, dp, ctypes.c_int64]
        L.orc_get_state.argtypes = [ctypes.c_void_p, dp, dp, dp, ctypes.POINTER(ctypes.c_int64)]
        L.orc_n_groups.restype = ctypes.c_int32
        L.orc_n_groups.argtypes = [ctypes.c_void_p]
        L.orc_group.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                                ctypes.POINTER(ctypes.c_int64),
                                ctypes.POINTER(ctypes.POINTER(ctypes.c_int32))]
        L.orc_accept_counts.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_int64)]
        L.orc_moments.argtypes = [ctypes.c_void_p, ctypes.c_int, dp, dp, ctypes.POINTER(ctypes.c_int64)]
        L.orc_split_rhat.restype = ctypes.c_double
        L.orc_split_rhat.argtypes = [dp, ctypes.c_int, ctypes.c_int64]
        L.orc_batch_means_mcse.restype = ctypes.c_double
        L.orc_batch_means_mcse.argtypes = [dp, ctypes.c_int64, ctypes.c_int64]
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_block_period.restype = ctypes.c_int32
        L.orc_block_period.argtypes = [ctypes.c_int32]
        L.orc_block_pass.restype = ctypes.c_int64
        L.orc_block_pass.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, dp, dp, ctypes.c_double,
                                     ctypes.c_double, dp, ctypes.POINTER(ctypes.c_uint8), dp,
                                     ctypes.POINTER(ctypes.c_int32)]
        L.orc_dirichlet_alpha.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
        L.orc_chunk_logprior.restype = ctypes.c_double
        L.orc_chunk_logprior.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# Stateless pieces
# ---------------------------------------------------------------------------

def philox(ctrs: np.ndarray, key0: int, key1: int) -> np.ndarray:
    """Philox4x32-10 of each 4-word counter row (uint32), key (key0, key1)."""
    c = np.ascontiguousarray(ctrs, dtype=np.uint32).reshape(-1, 4)
    out = np.empty_like(c)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    lib().orc_philox_many(c.ctypes.data_as(u32p), c.shape[0], key0 & 0xFFFFFFFF,
                          key1 & 0xFFFFFFFF, out.ctypes.data_as(u32p))
    return out


def normal(seed: int, m: int, t: int, chain: int, stream: int) -> float:
    return lib().orc_normal(seed, m, t, chain, stream)


def uniform(seed: int, m: int, t: int, chain: int, stream: int) -> float:
    return lib().orc_uniform(seed, m, t, chain, stream)


def loglik(w, G, o, sig, mu) -> np.ndarray:
    """Per-pixel log-likelihood log L_n(mu_n) (Eq. 6 factor), broadcast over inputs."""
    arrs = np.broadcast_arrays(*[np.asarray(v, np.float64) for v in (w, G, o, sig, mu)])
    flat = [_f64(a.ravel()) for a in arrs]
    out = np.empty(flat[0].shape, np.float64)
    lib().orc_loglik_many(*[_d(a) for a in flat], out.size, _d(out))
    return out.reshape(arrs[0].shape)


def loglik_emccd(w, G, o, sig, mu) -> np.ndarray:
    """Per-pixel log-likelihood of the EMCCD camera (orc_loglik_emccd: Poisson
    photoelectrons, Gamma(phi, 1) multiplication, read noise on the zero-photon
    reading), broadcast over inputs."""
    arrs = np.broadcast_arrays(*[np.asarray(v, np.float64) for v in (w, G, o, sig, mu)])
    flat = [_f64(a.ravel()) for a in arrs]
    out = np.empty(flat[0].shape, np.float64)
    lib().orc_loglik_emccd_many(*[_d(a) for a in flat], out.size, _d(out))
    return out.reshape(arrs[0].shape)


def forward(rho: np.ndarray, psf: np.ndarray) -> np.ndarray:
    """mu = P (x) rho with zero padding, same size (Eqs. 1-2).  PSF used as given."""
    rho = _f64(rho)
    psf = _f64(psf)
    mu = np.empty_like(rho)
    lib().orc_forward(_d(rho), rho.shape[0], rho.shape[1], _d(psf), psf.shape[0], _d(mu))
    return mu


def forward_sub(rho: np.ndarray, psf: np.ndarray, k: int) -> np.ndarray:
    """Pixel means over a finer object lattice (orc_forward_sub): rho [k H][k W]
    convolved with the PSF sampled on the object lattice (zero padding, same
    size), each pixel summing its k x k cells.  PSF used as given."""
    rho = _f64(rho)
    psf = _f64(psf)
    H, W = rho.shape[0] // k, rho.shape[1] // k
    assert rho.shape == (k * H, k * W)
    mu = np.empty((H, W))
    lib().orc_forward_sub(_d(rho), H, W, k, _d(psf), psf.shape[0], _d(mu))
    return mu


def dirichlet_alpha(psf: np.ndarray, th: int, tw: int) -> np.ndarray:
    """Concentration of the Dirichlet-OTF prior on a th x tw chunk: |OTF| of the
    PSF wrapped onto the chunk grid, normalised, floored at 1e-6 / K, renormalised."""
    psf = _f64(psf)
    out = np.empty(th * tw)
    lib().orc_dirichlet_alpha(_d(psf), psf.shape[0], th, tw, _d(out))
    return out.reshape(th, tw)


def chunk_logprior(rho: np.ndarray, alpha: np.ndarray) -> float:
    """log Dirichlet(|F(rho)| / sum |F(rho)|; alpha) of one chunk (Eqs. 7-8)."""
    rho = _f64(rho)
    a = _f64(alpha)
    return lib().orc_chunk_logprior(_d(rho), rho.shape[1], rho.shape[0], rho.shape[1], _d(a))


def split_rhat(x: np.ndarray) -> float:
    """Split-R-hat of draws x[chain, i]."""
    x = _f64(x)
    return lib().orc_split_rhat(_d(x), x.shape[0], x.shape[1])


def batch_means_mcse(x: np.ndarray, n_batches: int) -> float:
    x = _f64(x)
    return lib().orc_batch_means_mcse(_d(x), x.size, n_batches)


def set_threads(n: int) -> None:
    lib().orc_set_threads(n)


def max_threads() -> int:
    return lib().orc_max_threads()


# ---------------------------------------------------------------------------
# Sampler
# ---------------------------------------------------------------------------

class OracleSampler:
    """FP64 sampler over one frame, with the same schedule and RNG streams as the GPU."""

    def __init__(self, image, psf, gain, offset, sigma, *, n_chains: int = 1, seed: int = 0,
                 schedule: int = SCHED_CHROMATIC, block: int = 0, prior_kind: int = PRIOR_FLAT,
                 prior_a: float = 1.0, prior_b: float = 0.0, burn_in: int = 0,
                 log_step0: float = -1.5, camera: int = CAMERA_SCMOS, object_sub: int = 1):
        """object_sub = k > 1: rho lives on a (k H) x (k W) object lattice, each
        camera pixel integrating k x k cells, and the PSF is sampled on that
        lattice; state, draws and moments are object-lattice arrays, mu and the
        frame pixel-lattice ones."""
        image = _f64(image)
        H, W = image.shape
        s = psf.shape[0]
        g, o, sg = [_f64(np.broadcast_to(np.asarray(v, np.float64), (H, W))) for v in (gain, offset, sigma)]
        self.cfg = OrcConfig(H, W, s, n_chains, schedule, block, prior_kind, burn_in,
                             prior_a, prior_b, log_step0, seed & 0xFFFFFFFFFFFFFFFF, camera, object_sub)
        k = max(1, object_sub)
        self.H, self.W, self.C = H, W, n_chains
        self.Ho, self.Wo = k * H, k * W
        self._keep = (image, _f64(psf), g, o, sg)
        h = ctypes.c_void_p()
        rc = lib().orc_create(ctypes.byref(self.cfg), _d(self._keep[1]), _d(image), _d(g), _d(o),
                              _d(sg), ctypes.byref(h))
        if rc != OK:
            raise ValueError("oracle rejected the problem (code %d)" % rc)
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().orc_destroy(h)
            self._h = None

    def init(self, rho0: Optional[np.ndarray] = None) -> None:
        if rho0 is None:
            rc = lib().orc_init(self._h, None)
        else:
            r = _f64(np.broadcast_to(rho0, (self.C, self.Ho, self.Wo)))
            rc = lib().orc_init(self._h, _d(r))
        if rc != OK:
            raise ValueError("oracle init failed (code %d)" % rc)

    def sweep(self, n: int, trace: bool = False):
        tr = np.empty((n, self.C)) if trace else None
        lib().orc_sweeps(self._h, n, _d(tr) if trace else None)
        return tr

    def run_groups(self, t: int, g0: int, g1: int, refresh: bool = True, with_sabs: bool = False):
        """Run schedule groups [g0, g1) of sweep t; returns (delta, logu, accepted) maps
        (and sum_n |delta ell_n| per updated pixel when with_sabs), on the object lattice."""
        shp = (self.C, self.Ho, self.Wo)
        delta = np.full(shp, np.nan)
        logu = np.full(shp, np.nan)
        sabs = np.full(shp, np.nan)
        acc = np.full(shp, 255, np.uint8)
        rc = lib().orc_run_groups(self._h, t, g0, g1, int(refresh), _d(delta), _d(logu),
                                  acc.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), _d(sabs))
        if rc != OK:
            raise ValueError("bad group range")
        if with_sabs:
            return delta, logu, acc, sabs
        return delta, logu, acc

    def n_groups(self) -> int:
        return lib().orc_n_groups(self._h)

    def group(self, g: int) -> np.ndarray:
        b, e = ctypes.c_int64(), ctypes.c_int64()
        p = ctypes.POINTER(ctypes.c_int32)()
        lib().orc_group(self._h, g, ctypes.byref(b), ctypes.byref(e), ctypes.byref(p))
        return np.ctypeslib.as_array(p, shape=(self.Ho * self.Wo,))[b.value:e.value].copy()

    def set_state(self, rho, logstep, t: int) -> None:
        r = _f64(np.broadcast_to(rho, (self.C, self.Ho, self.Wo)))
        ls = _f64(np.broadcast_to(logstep, (self.C, self.Ho, self.Wo)))
        if lib().orc_set_state(self._h, _d(r), _d(ls), t) != OK:
            raise ValueError("invalid state")

    def state(self):
        shp = (self.C, self.Ho, self.Wo)
        rho, ls, mu = np.empty(shp), np.empty(shp), np.empty((self.C, self.H, self.W))
        t = ctypes.c_int64()
        lib().orc_get_state(self._h, _d(rho), _d(ls), _d(mu), ctypes.byref(t))
        return rho, ls, mu, t.value

    def log_posterior(self, chain: int = 0) -> float:
        return lib().orc_log_posterior(self._h, chain)

    def block_period(self) -> int:
        return lib().orc_block_period(self.cfg.s)

    def block_pass(self, pass_index: int, mean_log, sd_log, colour: int = -1, with_sabs: bool = False,
                   beta: float = 1.0, walk: float = 0.0):
        """One pass of the block move (or one colour of it): the reference move
        around (mean_log, sd_log) with AR coefficient beta, or, when walk > 0,
        the symmetric walk u' = u + walk (xi - P (x)_B xi) along what the blur
        removes (the maps are then unused).  Returns (accepted blocks, delta [C][blocks], accepted [C][blocks]) where
        the per-block records cover the last colour run (and the per-block sum of
        absolute terms when with_sabs)."""
        pm = _f64(np.broadcast_to(mean_log, (self.H, self.W)))
        ps = _f64(np.broadcast_to(sd_log, (self.H, self.W)))
        nmax = self.C * self.H * self.W
        delta = np.full(nmax, np.nan)
        sabs = np.full(nmax, np.nan)
        acc = np.full(nmax, 255, np.uint8)
        nb = ctypes.c_int32(0)
        a = lib().orc_block_pass(self._h, int(pass_index), int(colour), _d(pm), _d(ps), float(beta), float(walk),
                                 _d(delta),
                                 acc.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), _d(sabs), ctypes.byref(nb))
        n = nb.value
        out = (a, delta[:self.C * n].reshape(self.C, n), acc[:self.C * n].reshape(self.C, n))
        if with_sabs:
            out = out + (sabs[:self.C * n].reshape(self.C, n),)
        return out

    def accept_counts(self):
        a = np.zeros(self.C, np.int64)
        p = np.zeros(self.C, np.int64)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib().orc_accept_counts(self._h, a.ctypes.data_as(i64p), p.ctypes.data_as(i64p))
        return a, p

    def moments(self, chain: int = -1):
        mean = np.empty((self.Ho, self.Wo))
        var = np.empty((self.Ho, self.Wo))
        n = ctypes.c_int64()
        rc = lib().orc_moments(self._h, chain, _d(mean), _d(var), ctypes.byref(n))
        if rc != OK:
            raise ValueError("fewer than 2 samples")
        return mean, var, n.value
