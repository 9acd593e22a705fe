"""ctypes declarations of ``libbdc.so`` (the C ABI of ``include/bdc.h`` and
``include/bdc_unet.h``).

Argument marshalling only: every computation happens in the HIP library.
Loading fails loudly when the library has not been built.
"""

from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbdc.so")

BDC_OK, BDC_EINVAL, BDC_ENOMEM, BDC_EDEVICE, BDC_ESTATE, BDC_ENOTFINITE = 0, -1, -2, -3, -4, -5
BDC_SCHED_AUTO, BDC_SCHED_CHROMATIC, BDC_SCHED_BLOCK, BDC_SCHED_BLOCK_SERIES, BDC_SCHED_BLOCK9_SERIES = 0, 1, 2, 3, 4
BDC_CAMERA_SCMOS, BDC_CAMERA_EMCCD = 0, 1
BDC_PRIOR_FLAT, BDC_PRIOR_GAMMA, BDC_PRIOR_DIRICHLET = 0, 1, 2

STATUS_NAMES = {0: "BDC_OK", -1: "BDC_EINVAL", -2: "BDC_ENOMEM", -3: "BDC_EDEVICE",
                -4: "BDC_ESTATE", -5: "BDC_ENOTFINITE"}


class bdc_config(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int32), ("width", ctypes.c_int32),
                ("n_chains", ctypes.c_int32), ("prior_kind", ctypes.c_int32),
                ("prior_a", ctypes.c_float), ("prior_b", ctypes.c_float),
                ("burn_in", ctypes.c_int32), ("log_step0", ctypes.c_float),
                ("schedule", ctypes.c_int32), ("block_size", ctypes.c_int32),
                ("rhat_block", ctypes.c_int32), ("max_sweeps", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("camera", ctypes.c_int32), ("object_sub", ctypes.c_int32)]


class bdc_unet_config(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("base_channels", ctypes.c_int32),
                ("max_pixels", ctypes.c_int64), ("training", ctypes.c_int32)]


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_F32P = ctypes.POINTER(ctypes.c_float)

# name -> (restype, argtypes)
SIGNATURES = {
    "bdc_config_default": (None, [ctypes.POINTER(bdc_config)]),
    "bdc_create": (_I32, [ctypes.POINTER(bdc_config), _P, ctypes.POINTER(_P)]),
    "bdc_set_psf": (_I32, [_P, _P, _I32, _I32, _I32]),
    "bdc_set_camera_maps": (_I32, [_P, _P, _P, _P, _I32, _I32]),
    "bdc_init": (_I32, [_P, _P, _P, _I32]),
    "bdc_sweep": (_I32, [_P, _I32]),
    "bdc_posterior_moments": (_I32, [_P, _I32, _P, _P, ctypes.POINTER(_I64), _I32]),
    "bdc_rhat": (_I32, [_P, _F32P, _F32P]),
    "bdc_richardson_lucy": (_I32, [_P, _I32, _P, _I32]),
    "bdc_init_rl": (_I32, [_P, _I32]),
    "bdc_set_export": (_I32, [_P, _I32, _I32]),
    "bdc_samples": (_I32, [_P, _P, _I64, _I64, ctypes.POINTER(_I64), _I32]),
    "bdc_quantiles": (_I32, [_P, _P, _I32, _P, _I32]),
    "bdc_quantiles_of": (_I32, [_P, _I64, _I64, _P, _I32, _P, _P]),
    "bdc_cv_map": (_I32, [_P, _P, _I32]),
    "bdc_diag_window": (_I32, [ctypes.POINTER(bdc_config), _I64, _P, _P, _P, _P]),
    "bdc_rhat_map": (_I32, [_P, _P, _I32]),
    "bdc_window_mean": (_I32, [_P, _P, _I32]),
    "bdc_mcse": (_I32, [_P, _P, _I32]),
    "bdc_get_rho": (_I32, [_P, _P, _P, ctypes.POINTER(_I64), _I32]),
    "bdc_get_mu": (_I32, [_P, _P, _I32]),
    "bdc_loglik": (_I32, [_P, _I32, _P, _I32]),
    "bdc_logpost_trace": (_I32, [_P, _P, _I64, ctypes.POINTER(_I64)]),
    "bdc_accept_stats": (_I32, [_P, _P, _P]),
    "bdc_get_state": (_I32, [_P, _P, ctypes.POINTER(ctypes.c_size_t)]),
    "bdc_set_state": (_I32, [_P, _P, ctypes.c_size_t]),
    "bdc_set_rho": (_I32, [_P, _P, _P, _I64, _I32]),
    "bdc_debug_run_groups": (_I32, [_P, _I32, _I32, _P, _P, _I32]),
    "bdc_schedule_info": (_I32, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "bdc_profile": (_I32, [_P, _I32]),
    "bdc_profile_read": (_I32, [_P, _P, _P, _P]),
    "bdc_philox": (_I32, [_P, _I64, ctypes.c_uint32, ctypes.c_uint32, _P, _P]),
    "bdc_autotune": (_I32, [_P, _P, _I32, _I32, _P, ctypes.POINTER(_I32)]),
    "bdc_set_schedule": (_I32, [_P, _I32, _I32]),
    "bdc_batch_create": (_I32, [_P, _I32, _P, ctypes.POINTER(_P)]),
    "bdc_batch_sweep": (_I32, [_P, _I32]),
    "bdc_batch_check": (_I32, [_P]),
    "bdc_batch_info": (_I32, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "bdc_batch_last_error": (ctypes.c_char_p, [_P]),
    "bdc_batch_destroy": (None, [_P]),
    "bdc_unet_create": (_I32, [ctypes.POINTER(bdc_unet_config), _P, ctypes.POINTER(_P)]),
    "bdc_unet_param_count": (_I32, [_P, ctypes.POINTER(_I64)]),
    "bdc_unet_flops": (_I32, [_P, _I32, _I32, _I32, ctypes.POINTER(ctypes.c_double)]),
    "bdc_unet_set_params": (_I32, [_P, _P, _I32]),
    "bdc_unet_get_params": (_I32, [_P, _P, _I32]),
    "bdc_unet_forward": (_I32, [_P, _P, _I32, _I32, _I32, _P, _I32]),
    "bdc_unet_gradients": (_I32, [_P, _P, _P, _I32, _I32, _I32, _P, _F32P, _I32]),
    "bdc_unet_train_step": (_I32, [_P, _P, _P, _I32, _I32, _I32, ctypes.c_float, _F32P, _I32]),
    "bdc_unet_reset_optimizer": (_I32, [_P]),
    "bdc_debug_gemm_bf16": (_I32, [_P, _P, _P, _I64, _I32, _I32]),
    "bdc_unet_last_error": (ctypes.c_char_p, [_P]),
    "bdc_unet_destroy": (None, [_P]),
    "bdc_init_learned": (_I32, [_P, _P]),
    "bdc_set_block_proposal": (_I32, [_P, _P, _P, _I32]),
    "bdc_block_move": (_I32, [_P, _I32]),
    "bdc_set_block_beta": (_I32, [_P, ctypes.c_float]),
    "bdc_set_block_walk": (_I32, [_P, ctypes.c_float]),
    "bdc_block_stats": (_I32, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
    "bdc_debug_block_colour": (_I32, [_P, _I64, _I32, _P, _P, ctypes.POINTER(_I32)]),
    "bdc_training_targets": (_I32, [_P, _P, _P, _F32P, _I32]),
    "bdc_training_targets_noalloc": (_I32, [_P, _P, _P, _F32P, _I32]),
    "bdc_last_error": (ctypes.c_char_p, [_P]),
    "bdc_destroy": (None, [_P]),
}

_lib = None


def load():
    """Load libbdc.so and declare every entry point; raises if it is missing.

    torch (when installed) is imported first: it ships its own HIP runtime, and
    libbdc.so's dependency on libamdhip64.so.7 must resolve (by soname) to that
    already-loaded copy, so one process holds one runtime and torch's device
    pointers and streams are valid in the library.
    """
    global _lib
    if _lib is None:
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError("libbdc.so is not built (run __graft_entry__.build()); "
                              "the sampler has no CPU fallback")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib
