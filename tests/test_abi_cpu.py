"""Host-only checks of the C ABI: the library loads, exports every entry point
declared in include/*.h, and rejects bad configurations before touching a GPU."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bdc.h")
HEADERS = sorted(os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
                 if f.endswith(".h"))


def _declared():
    names = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(bdc_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_2411_00991_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        from paper_2411_00991_amd import build
        build.build()
    return _abi.load()


def test_header_declares_the_core_calls():
    names = _declared()
    for core in ("bdc_create", "bdc_set_psf", "bdc_set_camera_maps", "bdc_init", "bdc_sweep",
                 "bdc_posterior_moments", "bdc_destroy", "bdc_last_error", "bdc_unet_create",
                 "bdc_unet_forward", "bdc_unet_train_step", "bdc_init_learned", "bdc_block_move"):
        assert core in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_2411_00991_amd import _abi
    assert set(_declared()) == set(_abi.SIGNATURES)


def test_config_struct_layout_matches_header(lib):
    from paper_2411_00991_amd._abi import bdc_config
    assert ctypes.sizeof(bdc_config) == 64
    assert bdc_config.seed.offset == 48
    assert bdc_config.camera.offset == 56
    assert bdc_config.object_sub.offset == 60


def test_defaults(lib):
    import paper_2411_00991_amd as bdc
    cfg = bdc.bdc_config_default()
    assert cfg.n_chains == 1 and cfg.rhat_block == 25 and cfg.max_sweeps == 4096
    assert abs(cfg.log_step0 + 1.5) < 1e-7 and cfg.schedule == bdc.BDC_SCHED_AUTO
    assert cfg.camera == bdc.BDC_CAMERA_SCMOS


@pytest.mark.parametrize("field,value", [("height", 0), ("width", -3), ("n_chains", 0), ("n_chains", 65),
                                         ("prior_kind", 7), ("burn_in", -1), ("schedule", 9),
                                         ("block_size", -2), ("height", 40000), ("camera", 2),
                                         ("camera", -1), ("object_sub", 5), ("object_sub", -1)])
def test_create_rejects_bad_config_without_a_gpu(lib, field, value):
    import paper_2411_00991_amd as bdc
    cfg = bdc.bdc_config_default(height=16, width=16)
    setattr(cfg, field, value)
    with pytest.raises(bdc.BdcError) as ei:
        bdc.bdc_create(cfg)
    assert ei.value.status == bdc.BDC_EINVAL
    assert bdc.bdc_last_error(None) != "no error"


@pytest.mark.parametrize("fields", [dict(object_sub=2, schedule=3), dict(object_sub=3, schedule=4),
                                    dict(object_sub=2, prior_kind=2), dict(object_sub=4, height=4096, width=2049)])
def test_create_rejects_object_lattice_configs_without_a_gpu(lib, fields):
    """A finer object lattice runs the pixel-chromatic or block-phase scan
    (not the series scans) with a separable prior, within 2^27 object cells."""
    import paper_2411_00991_amd as bdc
    cfg = bdc.bdc_config_default(height=16, width=16)
    for k, v in fields.items():
        setattr(cfg, k, v)
    with pytest.raises(bdc.BdcError) as ei:
        bdc.bdc_create(cfg)
    assert ei.value.status == bdc.BDC_EINVAL


def test_create_rejects_frames_beyond_two_to_the_27_pixels(lib):
    import paper_2411_00991_amd as bdc
    cfg = bdc.bdc_config_default(height=16384, width=8193)       # 2^27 + 16384 pixels
    with pytest.raises(bdc.BdcError) as ei:
        bdc.bdc_create(cfg)
    assert ei.value.status == bdc.BDC_EINVAL and "2^27" in bdc.bdc_last_error(None)


def test_create_rejects_nonfinite_step(lib):
    import paper_2411_00991_amd as bdc
    cfg = bdc.bdc_config_default(height=16, width=16, log_step0=float("nan"))
    with pytest.raises(bdc.BdcError) as ei:
        bdc.bdc_create(cfg)
    assert ei.value.status == bdc.BDC_ENOTFINITE


def test_gamma_prior_needs_positive_shape(lib):
    import paper_2411_00991_amd as bdc
    cfg = bdc.bdc_config_default(height=16, width=16, prior_kind=bdc.BDC_PRIOR_GAMMA, prior_a=0.0)
    with pytest.raises(bdc.BdcError) as ei:
        bdc.bdc_create(cfg)
    assert ei.value.status == bdc.BDC_EINVAL


def test_null_arguments_are_errors_not_crashes(lib):
    assert lib.bdc_create(None, None, None) == -1
    assert lib.bdc_sweep(None, 1) == -1
    assert lib.bdc_last_error(None)
    lib.bdc_destroy(None)


def test_unet_create_rejects_bad_shapes(lib):
    from paper_2411_00991_amd._abi import bdc_unet_config
    out = ctypes.c_void_p()
    for lv, base, px in [(1, 32, 1 << 16), (7, 8, 1 << 20), (4, 12, 1 << 16), (4, 64, 1 << 16), (4, 32, 10)]:
        cfg = bdc_unet_config(levels=lv, base_channels=base, max_pixels=px, training=0)
        assert lib.bdc_unet_create(ctypes.byref(cfg), None, ctypes.byref(out)) == -1
        assert out.value is None
    assert lib.bdc_unet_create(None, None, ctypes.byref(out)) == -1


def test_gemm_hook_rejects_bad_sizes(lib):
    buf = (ctypes.c_uint16 * 64)()
    c = (ctypes.c_float * 64)()
    assert lib.bdc_debug_gemm_bf16(buf, buf, c, 4, 4, 6) == -1
    assert lib.bdc_debug_gemm_bf16(None, buf, c, 4, 4, 8) == -1


@pytest.mark.parametrize("rb,ms,burn", [(25, 4096, 0), (25, 4100, 60), (7, 100, 13), (10, 95, 0), (1, 5, 2)])
def test_diagnostic_windows_stay_inside_the_stores(lib, rb, ms, burn):
    """R-hat / window-mean batches [b_lo, b_lo + 2 half) and the trace entries
    they read lie inside the max_sweeps store for every t <= max_sweeps (also
    when max_sweeps is not a multiple of rhat_block); MCSE uses the complete
    post-burn-in batches; beyond max_sweeps the diagnostics refuse."""
    import paper_2411_00991_amd as bdc
    cfg = bdc.bdc_config_default(rhat_block=rb, max_sweeps=ms, burn_in=burn)
    for t in list(range(0, min(ms, 400) + 1)) + [ms - 1, ms]:
        b_lo, half, b0, nb = bdc.bdc_diag_window(cfg, t)
        done = t // rb
        assert half == done // 4 and b_lo + 2 * half == done
        assert (b_lo + 2 * half) * rb <= min(t, ms)          # trace [b_lo*rb, (b_lo+2h)*rb) stored
        assert b_lo + 2 * half <= ms // rb                     # batch store rows, all complete
        assert b0 == -(-burn // rb) and nb == max(done - b0, 0)
        assert b0 * rb >= burn                                  # MCSE batches are post-burn-in
    with pytest.raises(bdc.BdcError) as ei:
        bdc.bdc_diag_window(cfg, ms + 1)
    assert ei.value.status == bdc.BDC_ESTATE
