"""Pin of the truncation bound that the block-series scan relies on (CPU).

The pixel factor of the camera model (Image Formation Model, Eqs. 3-6),
sum_k exp(-a (k - c)^2) mu^k / k!, has only real negative zeros in mu (the
sequence exp(-a k^2) is a multiplier sequence, so the Polya-Schur theorem
applies to the image of exp).  Hence, with v = y / mu,

    ell(mu + y) - ell(mu) = -y + sum_{j>=1} h_j v^j,
    |sum_{j>J} h_j v^j| <= (E[phi] - Var[phi]) |v|^(J+1) / ((J+1)(1 - |v|)),

where E and Var are the photon-count posterior's moments at mu and the h_j
are the coefficients of log E[(1 + v)^phi].  This test builds the h_j here
from the explicit posterior (binomial moments, then the power-series
logarithm; NumPy/SciPy, FP64) and checks the oracle's exact ell against the
bound at J = 4 over many (c, a, mu, y), including the radius the kernel uses.
"""

import numpy as np
import pytest
from scipy.special import gammaln

import oracle

J = 4
G, O = 2.0, 100.0


def posterior(c, a, mu):
    """Photon-count posterior weights at mean mu over k = 0 .. kmax (FP64)."""
    kmax = int(max(c, mu, 0.0) + 60.0 * np.sqrt(max(c, mu, 1.0)) + 40.0 / np.sqrt(a) + 60)
    k = np.arange(0, kmax + 1, dtype=np.float64)
    lw = -a * (k - c) ** 2 - gammaln(k + 1) + k * np.log(mu)
    p = np.exp(lw - lw.max())
    return k, p / p.sum()


def taylor_coefficients(c, a, mu):
    """b_1..b_J of ell(mu + y) - ell(mu) in powers of y, and E - Var."""
    k, p = posterior(c, a, mu)
    # binomial moments E[C(phi, j)] about an integer shift k0 near the mean, so
    # the log-series sees numbers of the size of the posterior's spread
    k0 = float(np.floor((k * p).sum()))
    kk = k - k0
    s = [1.0]
    term = np.ones_like(kk)
    for j in range(1, J + 1):
        term = term * (kk - (j - 1)) / j
        s.append(float((term * p).sum()))
    # log(sum_j s_j v^j) as a power series (s_0 = 1)
    h = [0.0] * (J + 1)
    for j in range(1, J + 1):
        h[j] = s[j] - sum(i * h[i] * s[j - i] for i in range(1, j)) / j
    # + k0 log(1 + v)
    for j in range(1, J + 1):
        h[j] += k0 * (-1.0) ** (j + 1) / j
    b = [h[j] / mu ** j for j in range(1, J + 1)]
    b[0] -= 1.0
    mean = float((k * p).sum())
    var = float(((k - mean) ** 2 * p).sum())
    return np.array(b), mean - var


def ell(c, a, mu):
    sig = G / np.sqrt(2.0 * a)
    w = G * c + O
    mu = np.atleast_1d(np.asarray(mu, np.float64))
    return oracle.loglik(np.full(mu.shape, w), np.full(mu.shape, G), np.full(mu.shape, O),
                         np.full(mu.shape, sig), mu)


def bound(s2, v):
    v = np.abs(v)
    return s2 * v ** (J + 1) / ((J + 1) * (1.0 - v))


CASES = [
    # (c, a, mu): read noise from sharp (a = 30) to broad (a = 0.05), dim to bright, good and poor fits
    (0.3, 0.9, 0.7), (2.0, 0.9, 2.5), (13.0, 0.9, 12.0), (120.0, 0.9, 110.0), (800.0, 0.9, 820.0),
    (5.0, 0.05, 5.0), (60.0, 0.2, 55.0), (40.0, 6.0, 38.0), (250.0, 30.0, 250.0), (-1.5, 1.4, 0.4),
    (30.0, 2.0, 3.0), (3.0, 2.0, 30.0),
]


@pytest.mark.parametrize("c,a,mu", CASES)
def test_taylor_remainder_within_bound(c, a, mu):
    b, s2 = taylor_coefficients(c, a, mu)
    assert s2 >= -1e-9 * max(1.0, mu)          # E >= Var: the beta_i lie in (0, 1)
    s2 = max(s2, 0.0)
    v = np.concatenate([np.linspace(-0.5, 0.5, 41), [-0.01, 0.01, -0.002, 0.002]])
    v = v[v != 0.0]
    y = v * mu
    exact = ell(c, a, mu + y) - ell(c, a, mu)[0]
    series = sum(b[j] * y ** (j + 1) for j in range(J))
    err = np.abs(exact - series)
    # rounding of the two FP64 log-likelihoods (magnitude |ell|) on top of the bound
    slack = 1e-13 * (1.0 + np.abs(ell(c, a, mu)[0])) + 1e-12 * np.abs(exact)
    assert np.all(err <= bound(s2, v) * (1.0 + 1e-9) + slack), (err / (bound(s2, v) + slack)).max()


def test_bound_is_attained_for_sharp_read_noise():
    """Near-deterministic counts (Var -> 0) make every beta_i -> 1: the remainder
    approaches the bound, so the bound is not loose where it matters."""
    c, a, mu = 200.0, 40.0, 200.0
    b, s2 = taylor_coefficients(c, a, mu)
    v = -0.2
    err = abs((ell(c, a, mu * (1 + v)) - ell(c, a, mu))[0] - sum(b[j] * (v * mu) ** (j + 1) for j in range(J)))
    assert 0.5 * bound(s2, v) < err <= bound(s2, v) * (1.0 + 1e-9)


def test_radius_formula_keeps_error_below_tau():
    """The radius the kernel installs, u = min((2.5 tau / s2)^(1/5), 1/2) (1 - u0)^(1/5)
    with tau = 3e-9, keeps every evaluation inside it below tau / 2."""
    tau = 3e-9
    rng = np.random.default_rng(3)
    for _ in range(40):
        c = rng.uniform(-2.0, 400.0)
        a = float(np.exp(rng.uniform(np.log(0.05), np.log(30.0))))
        mu = float(np.exp(rng.uniform(np.log(0.1), np.log(500.0))))
        b, s2 = taylor_coefficients(c, a, mu)
        s2 = max(s2, 1e-30)
        u0 = min((2.5 * tau / s2) ** 0.2, 0.5)
        u = u0 * (1.0 - u0) ** 0.2
        assert bound(s2, u) <= 0.5 * tau * (1.0 + 1e-12)
        y = np.array([-u, -0.5 * u, 0.5 * u, u]) * mu
        exact = ell(c, a, mu + y) - ell(c, a, mu)[0]
        series = sum(b[j] * y ** (j + 1) for j in range(J))
        slack = 1e-13 * (1.0 + np.abs(ell(c, a, mu)[0]))
        assert np.all(np.abs(exact - series) <= 0.5 * tau + slack)
