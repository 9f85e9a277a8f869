"""ctypes mirror of include/gsr.h.  Argument marshalling only: every step of
the rasteriser runs in libgsr.so's HIP kernels."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsr.so")

GSR_OK, GSR_EINVAL, GSR_ENOMEM, GSR_ECAPACITY, GSR_EHIP, GSR_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
GSR_MAX_VIEWS = 64
GSR_ISOTROPIC, GSR_NO_GAUSS_GRADS, GSR_NO_POSE_GRADS, GSR_COUNT_WORK, GSR_PIXEL_HASH = 0x1, 0x2, 0x4, 0x8, 0x10
GSR_POSE_CENTRE, GSR_SYNC, GSR_DETERMINISTIC = 0x20, 0x40, 0x80
STAGES = ("binning", "blend_fwd", "blend_bwd", "project_bwd")

_fp = C.POINTER(C.c_float)
_vp = C.c_void_p


class Camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float)]


class Gaussians(C.Structure):
    _fields_ = [("n", C.c_int64), ("means", _vp), ("quats", _vp), ("log_scales", _vp),
                ("opacity_logits", _vp), ("rgb", _vp)]


class Views(C.Structure):
    _fields_ = [("n_views", C.c_int32), ("cams", C.POINTER(Camera)), ("quat", _vp), ("trans", _vp)]


class Options(C.Structure):
    _fields_ = [("w_rgb", C.c_float), ("w_depth", C.c_float), ("w_sil", C.c_float), ("w_prior", C.c_float),
                ("z_near", C.c_float), ("blur2d", C.c_float), ("sil_mask_thresh", C.c_float),
                ("tile_w", C.c_int32), ("tile_h", C.c_int32), ("flags", C.c_uint32)]


class Targets(C.Structure):
    _fields_ = [("rgb", _vp), ("depth", _vp), ("sil", _vp), ("prior", _vp), ("weight", _vp)]


class Images(C.Structure):
    _fields_ = [("rgb", _vp), ("depth", _vp), ("sil", _vp)]


class GaussGrads(C.Structure):
    _fields_ = [("means", _vp), ("quats", _vp), ("log_scales", _vp), ("opacity_logits", _vp), ("rgb", _vp)]


class PoseGrads(C.Structure):
    _fields_ = [("dq_t", _vp), ("dt", _vp), ("dq_c", _vp), ("dc", _vp)]


class Workspace(C.Structure):
    _fields_ = [("ptr", _vp), ("bytes", C.c_size_t), ("pair_capacity", C.c_int64)]


GSR_POSE_STATE_DOUBLES = 24


class PoseAdam(C.Structure):
    _fields_ = [("lr_rot", C.c_float), ("lr_pos", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float)]


class MapAdam(C.Structure):
    _fields_ = [("lr_means", C.c_float), ("lr_quats", C.c_float), ("lr_log_scales", C.c_float),
                ("lr_opacity", C.c_float), ("lr_rgb", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float)]


class GaussiansRW(C.Structure):
    _fields_ = [("n", C.c_int64), ("means", _vp), ("quats", _vp), ("log_scales", _vp),
                ("opacity_logits", _vp), ("rgb", _vp)]


EXPORTS = ["gsr_create", "gsr_destroy", "gsr_last_error", "gsr_workspace_size", "gsr_forward", "gsr_backward",
           "gsr_render_loss_grad", "gsr_read_counters", "gsr_read_work", "gsr_set_timing", "gsr_read_timing",
           "gsr_debug_binning", "gsr_debug_pixel_state", "gsr_selftest", "gsr_autotune", "gsr_set_tile",
           "gsr_graph_capture", "gsr_graph_launch", "gsr_graph_destroy", "gsr_pose_opt_init", "gsr_pose_opt_step",
           "gsr_track", "gsr_track_capture", "gsr_map_state_size", "gsr_map_opt_init", "gsr_map_opt_step",
           "gsr_densify_work_size", "gsr_densify", "gsr_map_iterate", "gsr_map_capture", "gsr_plan",
           "gsr_check_overflow", "gsr_render_loss_grad_noalloc"]

_lib = None


def load() -> C.CDLL:
    """Load libgsr.so.  Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -m paper_2408_05635_amd.build)")
    lib = C.CDLL(LIB_PATH)
    P = C.POINTER
    st = C.c_int
    lib.gsr_create.argtypes = [P(_vp), C.c_int]
    lib.gsr_create.restype = st
    lib.gsr_destroy.argtypes = [_vp]
    lib.gsr_destroy.restype = None
    lib.gsr_last_error.argtypes = [_vp]
    lib.gsr_last_error.restype = C.c_char_p
    lib.gsr_workspace_size.argtypes = [_vp, C.c_int64, P(Views), P(Options), C.c_int64, P(C.c_size_t)]
    lib.gsr_workspace_size.restype = st
    lib.gsr_forward.argtypes = [_vp, P(Gaussians), P(Views), P(Options), Workspace, Images, _vp]
    lib.gsr_forward.restype = st
    lib.gsr_backward.argtypes = [_vp, P(Gaussians), P(Views), P(Options), Workspace, Images, _vp, _vp, _vp,
                                 P(GaussGrads), P(PoseGrads), _vp]
    lib.gsr_backward.restype = st
    lib.gsr_render_loss_grad.argtypes = [_vp, P(Gaussians), P(Views), P(Options), P(Targets), Workspace, Images,
                                         _vp, P(GaussGrads), P(PoseGrads), _vp]
    lib.gsr_render_loss_grad.restype = st
    lib.gsr_render_loss_grad_noalloc.argtypes = [_vp, P(Gaussians), P(Views), P(Options), P(Targets), Images, _vp,
                                                 P(GaussGrads), P(PoseGrads), _vp, P(Workspace)]
    lib.gsr_render_loss_grad_noalloc.restype = st
    lib.gsr_read_counters.argtypes = [_vp, Workspace, _vp, P(C.c_int64), P(C.c_int64), P(C.c_int32)]
    lib.gsr_read_counters.restype = st
    lib.gsr_check_overflow.argtypes = [_vp, Workspace, _vp, P(C.c_int32)]
    lib.gsr_check_overflow.restype = st
    lib.gsr_plan.argtypes = [_vp, P(Gaussians), P(Views), P(Options), Workspace, P(C.c_int64), _vp]
    lib.gsr_plan.restype = st
    lib.gsr_read_work.argtypes = [_vp, Workspace, _vp, P(C.c_int64)]
    lib.gsr_read_work.restype = st
    lib.gsr_set_timing.argtypes = [_vp, C.c_int32]
    lib.gsr_set_timing.restype = st
    lib.gsr_read_timing.argtypes = [_vp, P(C.c_double), P(C.c_int64)]
    lib.gsr_read_timing.restype = st
    lib.gsr_debug_binning.argtypes = [_vp, P(Gaussians), P(Views), P(Options), Workspace, C.c_int64, C.c_int64,
                                      C.c_int64, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
    lib.gsr_debug_binning.restype = st
    lib.gsr_debug_pixel_state.argtypes = [_vp, P(Gaussians), P(Views), P(Options), Workspace, _vp, _vp, _vp, _vp]
    lib.gsr_debug_pixel_state.restype = st
    lib.gsr_autotune.argtypes = [_vp, P(Gaussians), P(Views), P(Options), P(Targets), Workspace, Images, _vp,
                                 P(GaussGrads), P(PoseGrads), C.c_int32, P(C.c_int32), P(C.c_double), _vp]
    lib.gsr_autotune.restype = st
    lib.gsr_set_tile.argtypes = [_vp, C.c_int64, P(Views), C.c_uint32, C.c_int32, C.c_int32]
    lib.gsr_set_tile.restype = st
    lib.gsr_graph_capture.argtypes = [_vp, P(Gaussians), P(Views), P(Options), P(Targets), Workspace, Images, _vp,
                                      P(GaussGrads), P(PoseGrads), _vp, P(C.c_int32)]
    lib.gsr_graph_capture.restype = st
    lib.gsr_graph_launch.argtypes = [_vp, C.c_int32, _vp]
    lib.gsr_graph_launch.restype = st
    lib.gsr_graph_destroy.argtypes = [_vp, C.c_int32]
    lib.gsr_graph_destroy.restype = st
    lib.gsr_selftest.argtypes = [_vp, _vp, _vp]
    lib.gsr_selftest.restype = st
    lib.gsr_pose_opt_init.argtypes = [_vp, C.c_int32, _vp, _vp, _vp, _vp]
    lib.gsr_pose_opt_init.restype = st
    lib.gsr_pose_opt_step.argtypes = [_vp, C.c_int32, _vp, _vp, P(PoseAdam), _vp, _vp, _vp, _vp]
    lib.gsr_pose_opt_step.restype = st
    track_args = [_vp, P(Gaussians), P(Camera), C.c_int32, _vp, _vp, P(Options), P(Targets), Workspace, Images, _vp,
                  P(PoseGrads), P(PoseAdam), _vp, C.c_int32, _vp, _vp]
    lib.gsr_track.argtypes = track_args
    lib.gsr_track.restype = st
    lib.gsr_track_capture.argtypes = track_args + [P(C.c_int32)]
    lib.gsr_track_capture.restype = st
    lib.gsr_map_state_size.argtypes = [C.c_int64, C.c_int32]
    lib.gsr_map_state_size.restype = C.c_size_t
    lib.gsr_map_opt_init.argtypes = [_vp, C.c_int64, C.c_int32, _vp, _vp]
    lib.gsr_map_opt_init.restype = st
    lib.gsr_map_opt_step.argtypes = [_vp, GaussiansRW, P(GaussGrads), C.c_int32, P(MapAdam), _vp, _vp]
    lib.gsr_map_opt_step.restype = st
    map_args = [_vp, GaussiansRW, P(Views), P(Options), P(Targets), Workspace, Images, _vp, P(GaussGrads), P(MapAdam),
                _vp, C.c_int32, _vp, _vp]
    lib.gsr_map_iterate.argtypes = map_args
    lib.gsr_map_iterate.restype = st
    lib.gsr_map_capture.argtypes = map_args + [P(C.c_int32)]
    lib.gsr_map_capture.restype = st
    lib.gsr_densify_work_size.argtypes = [C.c_int32, C.c_int32]
    lib.gsr_densify_work_size.restype = C.c_size_t
    lib.gsr_densify.argtypes = [_vp, Camera, _vp, _vp, _vp, _vp, _vp, C.c_float, GaussiansRW, C.c_int32, C.c_int64,
                                C.c_int64, _vp, _vp, C.c_size_t, _vp]
    lib.gsr_densify.restype = st
    _lib = lib
    return lib


class GsrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"gsr status {status}: {msg}")
        self.status = status


def check(status: int, ctx) -> None:
    if status != GSR_OK:
        msg = load().gsr_last_error(ctx)
        raise GsrError(status, msg.decode() if msg else "")
