"""ctypes binding of libfdgs.so (the C ABI in include/fdgs.h).

Argument marshalling only: every step of a render runs in the HIP kernels of
libfdgs.so.  If the library is missing, loading raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfdgs.so")

FDGS_OK = 0
FDGS_ERR_INVALID_ARG = 1
FDGS_ERR_HIP = 2
FDGS_ERR_CAPACITY = 3
FDGS_ERR_UNSUPPORTED = 4
FDGS_ERR_STATE = 5

MASK_TEMPORAL = 0
MASK_TEMPORAL_AND_TILE = 1
MASK_CONTRIBUTED = 2

EXPORTS = ["fdgs_last_error", "fdgs_version", "fdgs_create", "fdgs_destroy", "fdgs_render_cfg_default",
           "fdgs_slice_4d", "fdgs_build_active_mask", "fdgs_build_active_mask_noalloc", "fdgs_mask_overlap", "fdgs_measure_peaks", "fdgs_render_forward", "fdgs_render_backward",
           "fdgs_render_backward_2d", "fdgs_render_backward_params",
           "fdgs_state_release", "fdgs_state_binning", "fdgs_check_overflow", "fdgs_profile_enable",
           "fdgs_profile_read", "fdgs_render_batch", "fdgs_autotune", "fdgs_spatial_score",
           "fdgs_variation_score", "fdgs_prune", "fdgs_adam_step", "fdgs_sh_kmeans"]

STAGES = ["preprocess", "compact", "depth_sort", "offsets", "duplicate", "tile_sort", "ranges", "composite",
          "bwd_composite", "bwd_preprocess"]

c_float_p = ctypes.POINTER(ctypes.c_float)


class Model(ctypes.Structure):
    _fields_ = [("mean", ctypes.c_void_p), ("log_scale", ctypes.c_void_p), ("q_left", ctypes.c_void_p),
                ("q_right", ctypes.c_void_p), ("opacity_logit", ctypes.c_void_p), ("sh", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("sh_degree", ctypes.c_int32), ("sh_index", ctypes.c_void_p),
                ("sh_codebook", ctypes.c_void_p), ("sh_codebook_size", ctypes.c_int64)]


class Camera(ctypes.Structure):
    _fields_ = [("R", ctypes.c_double * 9), ("tvec", ctypes.c_double * 3), ("fx", ctypes.c_double),
                ("fy", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("znear", ctypes.c_double), ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class RenderCfg(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("pixels_per_thread", ctypes.c_int32), ("bg", ctypes.c_float * 3), ("alpha_min", ctypes.c_float), ("alpha_max", ctypes.c_float),
                ("t_min", ctypes.c_float), ("dilation", ctypes.c_float), ("temporal_cull", ctypes.c_int32),
                ("tile_cull", ctypes.c_int32), ("schedule", ctypes.c_int32), ("instance_capacity", ctypes.c_int64)]


class MaskSpec(ctypes.Structure):
    _fields_ = [("frame_times", ctypes.c_void_p), ("n_frames", ctypes.c_int32), ("views", ctypes.c_void_p),
                ("n_views", ctypes.c_int32), ("key_lo", ctypes.c_double), ("key_hi", ctypes.c_double),
                ("mode", ctypes.c_int32), ("alpha_min", ctypes.c_float), ("dilation", ctypes.c_float)]


class Grads(ctypes.Structure):
    _fields_ = [("mean", ctypes.c_void_p), ("log_scale", ctypes.c_void_p), ("q_left", ctypes.c_void_p),
                ("q_right", ctypes.c_void_p), ("opacity_logit", ctypes.c_void_p), ("sh", ctypes.c_void_p)]


class Binning(ctypes.Structure):
    _fields_ = [("sorted_ids", ctypes.c_void_p), ("tile_ranges", ctypes.c_void_p), ("rects", ctypes.c_void_p),
                ("depth", ctypes.c_void_p), ("visible", ctypes.c_void_p), ("n_inst", ctypes.c_int64),
                ("n_vis", ctypes.c_int64), ("n_proc", ctypes.c_int64), ("n_tiles", ctypes.c_int32),
                ("tiles_x", ctypes.c_int32), ("tiles_y", ctypes.c_int32)]


class View(ctypes.Structure):
    _fields_ = [("scene", ctypes.c_int32), ("cam", Camera), ("t", ctypes.c_double), ("idx", ctypes.c_void_p),
                ("n_idx", ctypes.c_int64)]


class TuneResult(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("pixels_per_thread", ctypes.c_int32), ("schedule", ctypes.c_int32), ("ms", ctypes.c_double),
                ("identical", ctypes.c_int32)]


class Profile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 10), ("calls", ctypes.c_int64 * 10), ("processed", ctypes.c_int64),
                ("visible", ctypes.c_int64), ("instances", ctypes.c_int64), ("pairs", ctypes.c_uint64),
                ("blended", ctypes.c_uint64)]


class FdgsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fdgs error {code}: {msg}")
        self.code = code


_LIB = None


def load() -> ctypes.CDLL:
    """Load libfdgs.so from the package directory (built by __graft_entry__.build())."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(LIB_PATH)
    P, I64, I32, D, VP = ctypes.POINTER, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p
    lib.fdgs_last_error.restype = ctypes.c_char_p
    lib.fdgs_version.restype = ctypes.c_char_p
    lib.fdgs_create.argtypes = [P(VP), I32]
    lib.fdgs_destroy.argtypes = [VP]
    lib.fdgs_render_cfg_default.argtypes = [P(RenderCfg)]
    lib.fdgs_render_cfg_default.restype = None
    lib.fdgs_slice_4d.argtypes = [VP, P(Model), D, VP, I64, VP, VP, VP, VP]
    lib.fdgs_build_active_mask.argtypes = [VP, P(Model), P(MaskSpec), VP, VP, VP, VP]
    lib.fdgs_build_active_mask_noalloc.argtypes = [P(Model), P(MaskSpec), VP, VP, VP, VP]
    lib.fdgs_mask_overlap.argtypes = [VP, VP, I64, VP, VP]
    lib.fdgs_measure_peaks.argtypes = [VP, P(D), VP]
    lib.fdgs_render_forward.argtypes = [VP, P(Model), VP, VP, P(Camera), D, P(RenderCfg), VP, VP, P(VP), VP]
    lib.fdgs_render_backward.argtypes = [VP, VP, VP, P(Grads), VP]
    lib.fdgs_render_backward_2d.argtypes = [VP, VP, VP, VP]
    lib.fdgs_render_backward_params.argtypes = [VP, VP, P(Grads), VP]
    lib.fdgs_state_release.argtypes = [VP, VP]
    lib.fdgs_state_binning.argtypes = [VP, VP, P(Binning), VP]
    lib.fdgs_check_overflow.argtypes = [VP, VP]
    lib.fdgs_profile_enable.argtypes = [VP, I32]
    lib.fdgs_profile_read.argtypes = [VP, P(Profile), I32]
    lib.fdgs_render_batch.argtypes = [VP, P(Model), I32, P(View), I32, P(RenderCfg), I32, I32, VP, VP]
    lib.fdgs_autotune.argtypes = [VP, P(Model), I32, P(View), I32, I32, I32, P(RenderCfg), P(TuneResult), I32,
                                  P(I32), VP]
    for name in EXPORTS:
        f = getattr(lib, name)
        if f.restype is ctypes.c_int:   # default restype: status
            f.restype = ctypes.c_int32
    _LIB = lib
    return lib


def check(status: int) -> None:
    if status != FDGS_OK:
        raise FdgsError(status, load().fdgs_last_error().decode())


def default_cfg(**kw) -> RenderCfg:
    cfg = RenderCfg()
    load().fdgs_render_cfg_default(ctypes.byref(cfg))
    for k, v in kw.items():
        if k == "bg":
            for i in range(3):
                cfg.bg[i] = float(v[i])
        else:
            setattr(cfg, k, v)
    return cfg


def camera_struct(cam) -> Camera:
    """From any object with R (3x3), tvec (3), fx, fy, cx, cy, width, height, znear."""
    c = Camera()
    R = [float(x) for row in cam.R for x in row]
    for i in range(9):
        c.R[i] = R[i]
    for i in range(3):
        c.tvec[i] = float(cam.tvec[i])
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.znear = float(cam.znear)
    c.width, c.height = int(cam.width), int(cam.height)
    return c
