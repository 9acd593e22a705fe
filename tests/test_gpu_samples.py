"""Thinned sample export, per-pixel quantiles and the CV map (Results, "Our
package" and "Uncertainty": many candidate deconvolved images, their
quantiles, variance and coefficient of variation).

Quantiles are checked against numpy.quantile (its default linear
interpolation between order statistics), exactly where the level falls on an
order statistic; the exported samples against the chain states read after
every sweep, bit for bit; the CV map against sqrt(var) / mean of the pooled
moments.
"""

import numpy as np
import pytest

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


@pytest.mark.parametrize("n,n_pix", [(1, 7), (2, 130), (101, 333), (400, 1000), (1000, 77), (4096, 65)])
def test_quantiles_of_seeded_data_match_numpy(bdc, n, n_pix):
    import torch
    say("quantiles of seeded data, n = %d, %d pixels" % (n, n_pix))
    rng = np.random.default_rng(n + n_pix)
    x = rng.gamma(2.0, 3.0, (n, n_pix)).astype(np.float32)
    x[:, ::5] = np.round(x[:, ::5])                    # ties
    probs = np.array([0.0, 0.025, 0.1, 0.25, 0.5, 0.75, 0.9, 0.975, 1.0], np.float32)
    out = torch.empty((len(probs), n_pix), dtype=torch.float32, device="cuda")
    bdc.bdc_quantiles_of(torch.from_numpy(x).cuda(), torch.from_numpy(probs).cuda(), out)
    got = out.cpu().numpy()
    xs = np.sort(x.astype(np.float64), axis=0)
    for q, p in enumerate(probs.astype(np.float64)):
        h = (n - 1) * p
        lo = int(np.floor(h))
        want = xs[lo] if lo + 1 >= n else xs[lo] + (h - lo) * (xs[lo + 1] - xs[lo])
        np.testing.assert_allclose(got[q], want, rtol=1e-6, atol=1e-6)
        np.testing.assert_allclose(got[q], np.quantile(x.astype(np.float64), p, axis=0), rtol=1e-6, atol=1e-6)
        if h == lo:                                     # an order statistic: exact
            assert np.array_equal(got[q], xs[lo].astype(np.float32))
    assert np.array_equal(got[0], x.min(axis=0)) and np.array_equal(got[-1], x.max(axis=0))


def test_export_quantiles_and_cv_on_a_sampler(bdc):
    say("thinned export, quantiles and CV of a sampler run")
    fr = synth.frame_beads_segments(40, seed=3, n_prims=8, psf=synth.gaussian_psf(1.2, 7))
    H, W = fr.image.shape
    C, burn, thin, cap = 3, 5, 3, 10
    S = bdc.Sampler(np.asarray(fr.psf, np.float32), np.float32(2.0), np.float32(100.0), np.float32(1.5),
                    height=H, width=W, n_chains=C, seed=9, burn_in=burn)
    S.set_export(thin, cap)
    S.init(np.asarray(fr.image, np.float32))
    want = []
    for t in range(40):
        S.sweep(1)
        if t >= burn and (t - burn) % thin == 0 and len(want) < cap:
            want.append(S.rho()[0])
    got = S.samples()
    assert got.shape == (cap, C, H, W)
    assert np.array_equal(got, np.array(want))
    probs = [0.05, 0.25, 0.5, 0.75, 0.95]
    q = S.quantiles(probs)
    pooled = got.reshape(cap * C, H, W).astype(np.float64)
    np.testing.assert_allclose(q, np.quantile(pooled, probs, axis=0), rtol=1e-6, atol=1e-6)
    # n = 30 values: level 0.5 falls between order statistics 14 and 15; the
    # extremes are order statistics
    q01 = S.quantiles([0.0, 1.0])
    assert np.array_equal(q01[0], got.min(axis=(0, 1))) and np.array_equal(q01[1], got.max(axis=(0, 1)))
    m, v, _ = S.moments()
    cv = S.cv_map()
    np.testing.assert_allclose(cv, np.sqrt(v.astype(np.float64)) / m, rtol=2e-6)
    S.set_export(0, 0)
    assert S.samples().shape[0] == 0
    S.close()


def test_export_refused_after_burn_in(bdc):
    fr = synth.frame_beads_segments(24, seed=4, n_prims=4, psf=synth.gaussian_psf(1.2, 7))
    S = bdc.Sampler(np.asarray(fr.psf, np.float32), np.float32(2.0), np.float32(100.0), np.float32(1.5),
                    height=24, width=24, burn_in=2)
    S.init(np.asarray(fr.image, np.float32))
    S.sweep(3)
    with pytest.raises(bdc.BdcError) as ei:
        S.set_export(1, 4)
    assert ei.value.status == bdc.BDC_ESTATE
    with pytest.raises(bdc.BdcError) as ei:
        S.quantiles([0.5])
    assert ei.value.status == bdc.BDC_ESTATE
    S.close()
