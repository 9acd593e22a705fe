"""The allocation-free variant of bdc_training_targets, through the C ABI:
its outputs equal those of bdc_training_targets bit for bit, on two calls in a
row (the second on a smaller frame, reusing the library's scratch array), for
host and device outputs; frames beyond its scratch are refused."""

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


def _sampler(bdc, n, seed):
    fr = synth.frame_beads_segments(n, seed=seed, n_prims=6, psf=synth.gaussian_psf(1.2, 7))
    g, o, s = [np.asarray(a, np.float32) for a in fr.camera.maps(n, n)]
    S = bdc.Sampler(np.asarray(fr.psf, np.float32), g, o, s, height=n, width=n, n_chains=2, seed=seed, burn_in=3)
    S.init(np.asarray(fr.image, np.float32))
    S.sweep(8)
    return S


def test_noalloc_training_targets_match_the_allocating_call(bdc):
    import torch
    for n, seed in ((48, 1), (24, 2)):                       # second call: a smaller frame
        say("frame %d x %d" % (n, n))
        S = _sampler(bdc, n, seed)
        x0 = np.empty((n, n), np.float32)
        t0 = np.empty((n, n, 2), np.float32)
        sc0 = bdc.bdc_training_targets(S.ctx, x0, t0)
        x1 = np.full((n, n), np.nan, np.float32)
        t1 = np.full((n, n, 2), np.nan, np.float32)
        sc1 = bdc.bdc_training_targets_noalloc(S.ctx, x1, t1)
        assert sc1 == sc0
        assert np.array_equal(x1, x0) and np.array_equal(t1, t0)
        xd = torch.full((n, n), float("nan"), device="cuda")
        td = torch.full((n, n, 2), float("nan"), device="cuda")
        sc2 = bdc.bdc_training_targets_noalloc(S.ctx, xd, td)
        torch.cuda.synchronize()
        assert sc2 == sc0
        assert np.array_equal(xd.cpu().numpy(), x0) and np.array_equal(td.cpu().numpy(), t0)
        S.close()


def test_noalloc_training_targets_refuse_frames_beyond_the_scratch(bdc):
    n = 2400                                                   # 5.76 M pixels > 5,592,384
    psf = synth.gaussian_psf(0.8, 3).astype(np.float32)
    S = bdc.Sampler(psf, np.float32(2.0), np.float32(100.0), np.float32(1.5), height=n, width=n, burn_in=0,
                    max_sweeps=8)
    S.init(np.full((n, n), 110.0, np.float32))
    S.sweep(2)
    x = np.empty((n, n), np.float32)
    t = np.empty((n, n, 2), np.float32)
    with pytest.raises(bdc.BdcError) as ei:
        bdc.bdc_training_targets_noalloc(S.ctx, x, t)
    assert ei.value.status == bdc.BDC_EINVAL
    S.close()
