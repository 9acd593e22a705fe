"""Richardson-Lucy deconvolution in FP64 -- TEST INFRASTRUCTURE ONLY.

Only the test-suite and the benchmark's CPU-baseline leg may import this
module.  It shares no code with the GPU library.

The paper's comparison method (Introduction; Results, Simulated Data): the
multiplicative expectation-maximisation update for Poisson counts d blurred by
the PSF P (Richardson 1972; Lucy 1974), with the image formation of Methods,
Eqs. 1-2 (same-size convolution, object zero outside the frame):

    rho_{k+1}(m) = rho_k(m) * sum_n P[n - m] d_n / mu_n(rho_k)  /  sum_n P[n - m],
    mu(rho) = P (x) rho,

the sums over the pixels n of the frame (the last factor, P^T applied to an
image of ones, is below 1 near the frame's edge).  d is the photon image
max((w - o) / G, 0) of an sCMOS frame; rho_0 is the mean of d everywhere.
A pixel with mu_n = 0 contributes nothing.  The convolutions use
scipy.signal.convolve2d (a library primitive).
"""

from __future__ import annotations

import numpy as np
from scipy import signal


def photon_image(w, gain, offset):
    return np.maximum((np.asarray(w, np.float64) - offset) / gain, 0.0)


def _conv(x, psf):
    return signal.convolve2d(x, psf, mode="same", boundary="fill", fillvalue=0.0)


def _corr(x, psf):
    return signal.convolve2d(x, psf[::-1, ::-1], mode="same", boundary="fill", fillvalue=0.0)


def richardson_lucy(d, psf, n_iter, rho0=None):
    """n_iter Richardson-Lucy iterations from rho0 (default: mean(d) everywhere).
    Returns rho (FP64)."""
    d = np.asarray(d, np.float64)
    psf = np.asarray(psf, np.float64)
    psf = psf / psf.sum()
    rho = np.full(d.shape, d.mean()) if rho0 is None else np.asarray(rho0, np.float64).copy()
    norm = _corr(np.ones_like(d), psf)
    for _ in range(n_iter):
        mu = _conv(rho, psf)
        q = np.where(mu > 0, d / np.where(mu > 0, mu, 1.0), 0.0)
        rho = rho * _corr(q, psf) / norm
    return rho


def poisson_loglik(d, rho, psf):
    """sum_n d_n log mu_n - mu_n (the Poisson log-likelihood RL ascends, up to a constant)."""
    psf = np.asarray(psf, np.float64) / np.sum(psf)
    mu = _conv(np.asarray(rho, np.float64), psf)
    d = np.asarray(d, np.float64)
    return float(np.sum(np.where(d > 0, d * np.log(np.maximum(mu, 1e-300)), 0.0) - mu))
