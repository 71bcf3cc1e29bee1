"""ctypes declarations of the C ABI in include/gsr.h (argument marshalling only).

The library is loaded from this package directory.  torch is imported first so
the renderer shares torch's HIP runtime (both resolve libamdhip64.so.7 to the
same loaded copy) and can use torch's device memory and streams directly.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must be loaded before libgsr.so, see above)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgsr.so")

c_float_p = ctypes.POINTER(ctypes.c_float)
c_int32_p = ctypes.POINTER(ctypes.c_int32)
c_uint8_p = ctypes.POINTER(ctypes.c_uint8)
c_void_p = ctypes.c_void_p

GSR_OK = 0
GSR_E_INVALID = -1
GSR_E_CAPACITY = -2
GSR_E_HIP = -3
GSR_E_UNSUPPORTED = -4
GSR_E_STATE = -5

GSR_FULL_RECT = 1 << 0
GSR_GAUSS_GRAD = 1 << 1
GSR_POSE_GRAD = 1 << 2
GSR_PAPER_POSE_APPROX = 1 << 3
GSR_GRAD_OVERWRITE = 1 << 4

GSR_NOALLOC_SCRATCH_BYTES = 64 << 20


class gsr_camera(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("R", ctypes.c_float * 9), ("t", ctypes.c_float * 3), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("_pad", ctypes.c_int32 * 2)]


class gsr_gaussians(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("mean", c_void_p), ("log_scale", c_void_p), ("quat", c_void_p),
                ("opacity_logit", c_void_p), ("rgb", c_void_p), ("mask", c_void_p), ("sh", c_void_p)]


class gsr_config(ctypes.Structure):
    _fields_ = [("alpha_min", ctypes.c_float), ("alpha_max", ctypes.c_float), ("T_min", ctypes.c_float),
                ("cutoff_sigma", ctypes.c_float), ("z_near", ctypes.c_float), ("lowpass", ctypes.c_float),
                ("bg", ctypes.c_float * 3), ("flags", ctypes.c_uint32), ("fov_guard", ctypes.c_float)]


class gsr_images(ctypes.Structure):
    _fields_ = [("rgb", c_void_p), ("depth", c_void_p), ("T_final", c_void_p), ("last", c_void_p),
                ("loss", c_void_p)]


class gsr_grads(ctypes.Structure):
    _fields_ = [("d_mean", c_void_p), ("d_log_scale", c_void_p), ("d_quat", c_void_p),
                ("d_opacity_logit", c_void_p), ("d_rgb", c_void_p), ("d_pose", c_void_p), ("d_sh", c_void_p)]


class gsr_tuning(ctypes.Structure):
    _fields_ = [("blocks_per_cu", ctypes.c_int32), ("tiles_per_pop", ctypes.c_int32),
                ("lpt_order", ctypes.c_int32), ("batch", ctypes.c_int32)]


class gsr_gaussians_out(ctypes.Structure):
    _fields_ = [("mean", c_void_p), ("log_scale", c_void_p), ("quat", c_void_p), ("opacity_logit", c_void_p),
                ("rgb", c_void_p), ("sh", c_void_p)]


class gsr_expand_params(ctypes.Structure):
    _fields_ = [("tau_T", ctypes.c_float), ("tau_D", ctypes.c_float), ("scale_factor", ctypes.c_float),
                ("opacity_logit_init", ctypes.c_float)]


assert ctypes.sizeof(gsr_camera) == 80
assert ctypes.sizeof(gsr_config) == 44

_P = ctypes.POINTER
# name -> (restype, argtypes)
SIGNATURES = {
    "gsr_default_config": (gsr_config, []),
    "gsr_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "gsr_last_error": (ctypes.c_char_p, [c_void_p]),
    "gsr_create": (ctypes.c_int, [ctypes.c_int, _P(c_void_p)]),
    "gsr_destroy": (None, [c_void_p]),
    "gsr_plan": (ctypes.c_int, [c_void_p, ctypes.c_int64, ctypes.c_int, c_int32_p, ctypes.c_int64,
                                _P(ctypes.c_size_t)]),
    "gsr_render_forward": (ctypes.c_int, [c_void_p, _P(gsr_gaussians), c_void_p, ctypes.c_int, _P(gsr_config),
                                          c_void_p, ctypes.c_size_t, _P(gsr_images), c_void_p]),
    "gsr_forward_generation": (ctypes.c_int64, [c_void_p]),
    "gsr_render_backward": (ctypes.c_int, [c_void_p, _P(gsr_gaussians), c_void_p, ctypes.c_int, _P(gsr_config),
                                           c_void_p, ctypes.c_size_t, ctypes.c_int64, c_void_p, c_void_p, c_void_p,
                                           _P(gsr_grads), c_void_p]),
    "gsr_l1_loss_grad": (ctypes.c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                        ctypes.c_float, ctypes.c_float, c_void_p, c_void_p, c_void_p, c_void_p,
                                        c_void_p]),
    "gsr_loss_median": (ctypes.c_int, [c_void_p, c_void_p, c_void_p, ctypes.c_float, c_void_p, c_void_p]),
    "gsr_render_l1_fused": (ctypes.c_int, [c_void_p, _P(gsr_gaussians), c_void_p, ctypes.c_int, _P(gsr_config),
                                           c_void_p, c_void_p, c_void_p, ctypes.c_float, ctypes.c_float, c_void_p,
                                           c_void_p, ctypes.c_size_t, _P(gsr_images), _P(gsr_grads), c_void_p,
                                           c_void_p]),
    "gsr_render_l1_fused_noalloc": (ctypes.c_int, [c_void_p, _P(gsr_gaussians), c_void_p, ctypes.c_int,
                                                   _P(gsr_config), c_void_p, c_void_p, c_void_p, ctypes.c_float,
                                                   ctypes.c_float, c_void_p, _P(gsr_images), _P(gsr_grads),
                                                   c_void_p, c_void_p]),
    "gsr_graph_capture": (ctypes.c_int, [c_void_p, _P(gsr_gaussians), c_void_p, ctypes.c_int, _P(gsr_config),
                                         c_void_p, c_void_p, c_void_p, ctypes.c_float, ctypes.c_float, c_void_p,
                                         c_void_p, ctypes.c_size_t, _P(gsr_images), _P(gsr_grads), c_void_p,
                                         c_void_p]),
    "gsr_graph_launch": (ctypes.c_int, [c_void_p, c_void_p]),
    "gsr_check_overflow": (ctypes.c_int, [c_void_p, c_void_p, c_void_p]),
    "gsr_required_pairs": (ctypes.c_int64, [c_void_p]),
    "gsr_pair_count": (ctypes.c_int64, [c_void_p, c_void_p, c_void_p]),
    "gsr_debug_tiles": (ctypes.c_int, [c_void_p, c_void_p, _P(c_void_p), _P(c_void_p), _P(ctypes.c_int64)]),
    "gsr_get_tuning": (ctypes.c_int, [c_void_p, _P(gsr_tuning)]),
    "gsr_set_tuning": (ctypes.c_int, [c_void_p, _P(gsr_tuning)]),
    "gsr_autotune": (ctypes.c_int, [c_void_p, _P(gsr_gaussians), c_void_p, ctypes.c_int, _P(gsr_config),
                                    c_void_p, c_void_p, c_void_p, ctypes.c_float, ctypes.c_float, c_void_p,
                                    ctypes.c_size_t, _P(gsr_grads), c_void_p, ctypes.c_int, _P(gsr_tuning),
                                    c_void_p]),
    "gsr_select_reliable": (ctypes.c_int, [c_void_p, _P(gsr_gaussians), c_void_p, c_void_p, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_float, ctypes.c_float, c_void_p, c_void_p]),
    "gsr_expand_add": (ctypes.c_int, [c_void_p, c_void_p, ctypes.c_int, c_void_p, c_void_p, c_void_p, c_void_p,
                                      _P(gsr_expand_params), c_void_p, ctypes.c_size_t, ctypes.c_int64,
                                      ctypes.c_int64, _P(gsr_gaussians_out), c_void_p, c_void_p, c_void_p]),
    "gsr_expand_delete": (ctypes.c_int, [c_void_p, _P(gsr_gaussians), c_void_p, c_void_p, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_float, ctypes.c_float, ctypes.c_float, c_void_p,
                                         c_void_p, c_void_p]),
    "gsr_pose_apply": (ctypes.c_int, [c_void_p, ctypes.c_int, c_void_p, c_void_p, c_void_p, c_void_p]),
    "gsr_pose_xi_grad": (ctypes.c_int, [c_void_p, ctypes.c_int, c_void_p, c_void_p, c_void_p, c_void_p]),
    "gsr_pose_from_qt": (ctypes.c_int, [c_void_p, ctypes.c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "gsr_pose_qt_grad": (ctypes.c_int, [c_void_p, ctypes.c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                        c_void_p]),
    "gsr_set_profiling": (ctypes.c_int, [c_void_p, ctypes.c_int]),
    "gsr_stage_times": (ctypes.c_int, [c_void_p, _P(ctypes.c_double), _P(ctypes.c_int64)]),
    "gsr_work_counts": (ctypes.c_int, [c_void_p, _P(gsr_gaussians), _P(gsr_config), c_void_p, c_void_p,
                                        _P(ctypes.c_int64)]),
}

STAGES = ("preprocess", "depth_sort", "emit", "pair_sort", "ranges", "raster", "raster_bwd", "pregrad")

_LIB = None


def load():
    """Load libgsr.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2311_11700_amd.build` "
                           "(or __graft_entry__.build()); there is no fallback renderer")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def exported_symbols():
    return list(SIGNATURES)
