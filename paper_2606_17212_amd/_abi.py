"""ctypes view of the C ABI in ``include/dgs.h`` (argument marshalling only).

The library is the in-tree ``libdgs.so`` built by ``paper_2606_17212_amd.build``.
There is no fallback: if the library is missing or fails to load, every
entry point raises.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdgs.so")

DGS_OK = 0
DGS_ERR_OVERFLOW = 3

EXPORTS = (
    "dgs_abi_version", "dgs_status_string", "dgs_last_error", "dgs_workspace_bytes",
    "dgs_count_instances", "dgs_render", "dgs_render_per_state", "dgs_render_psnr",
    "dgs_backward", "dgs_check", "dgs_workspace_sections", "dgs_bin", "dgs_composite",
    "dgs_composite_psnr", "dgs_composite_stats", "dgs_composite_launch", "dgs_utility_workspace_bytes",
    "dgs_utility_count", "dgs_utility", "dgs_utility_check", "dgs_distortion_scratch_bytes", "dgs_distortion",
    "dgs_risk_adjusted", "dgs_sample_states", "dgs_objective_scratch_bytes", "dgs_objective",
    "dgs_objective_check", "dgs_l1_scratch_bytes", "dgs_l1_loss", "dgs_l1_loss_grad",
    "dgs_probe_copy", "dgs_probe_valu", "dgs_render_noalloc",
)
NOALLOC_SCRATCH_BYTES = 64 << 20  # DGS_NOALLOC_SCRATCH_BYTES
PROBE_THREADS = 524288


class Scene(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("rank", ctypes.c_int32), ("sh_degree", ctypes.c_int32),
                ("num_clusters", ctypes.c_int32), ("num_contexts", ctypes.c_int32),
                ("mean", ctypes.c_void_p), ("log_scale", ctypes.c_void_p), ("quat", ctypes.c_void_p),
                ("opacity_logit", ctypes.c_void_p), ("color", ctypes.c_void_p),
                ("temporal", ctypes.c_void_p), ("packet_layer", ctypes.c_void_p),
                ("cluster_affine", ctypes.c_void_p), ("refine", ctypes.c_void_p)]


class ObjectiveWeights(ctypes.Structure):
    _fields_ = [("lambda_ssim", ctypes.c_float), ("lambda_c", ctypes.c_float), ("alpha", ctypes.c_float),
                ("lambda_t", ctypes.c_float), ("lambda_m", ctypes.c_float), ("lambda_a", ctypes.c_float)]


class Camera(ctypes.Structure):
    _fields_ = [("R_cw", ctypes.c_float * 9), ("t_cw", ctypes.c_float * 3), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("near_z", ctypes.c_float), ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class States(ctypes.Structure):
    _fields_ = [("num_states", ctypes.c_int32), ("codes", ctypes.c_void_p),
                ("basis", ctypes.c_float * 4), ("background", ctypes.c_float * 3)]


TUNE_PERSISTENT = 1  # dgs_tuning.flags: persistent compositing launch
TUNE_GRID = 2        # dgs_tuning.flags: one workgroup per work item (0 = automatic)


class Tuning(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("states_per_group", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("lds_batch", ctypes.c_int32)]


class SceneGrad(ctypes.Structure):
    _fields_ = [("mean", ctypes.c_void_p), ("log_scale", ctypes.c_void_p), ("quat", ctypes.c_void_p),
                ("opacity_logit", ctypes.c_void_p), ("color", ctypes.c_void_p),
                ("temporal", ctypes.c_void_p), ("refine", ctypes.c_void_p)]


class WorkspaceView(ctypes.Structure):
    _fields_ = [("rec0", ctypes.c_uint64), ("rec1", ctypes.c_uint64), ("rec2", ctypes.c_uint64),
                ("rect", ctypes.c_uint64), ("ranges", ctypes.c_uint64), ("sorted_ids", ctypes.c_uint64),
                ("tiles_x", ctypes.c_int32), ("tiles_y", ctypes.c_int32)]


ABI_VERSION = 3  # the structs below match include/dgs.h of this version


class DgsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"dgs status {status}: {message}")
        self.status = status


_lib = None


def lib():
    """Load ``libdgs.so`` (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2606_17212_amd/build.py "
                          "(or __graft_entry__.build()) first")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    L.dgs_abi_version.restype = ctypes.c_int
    if L.dgs_abi_version() != ABI_VERSION:
        raise ImportError(f"{LIB_PATH} has ABI version {L.dgs_abi_version()}, the binding expects "
                          f"{ABI_VERSION}; rebuild it")
    L.dgs_status_string.restype = ctypes.c_char_p
    L.dgs_status_string.argtypes = [ctypes.c_int]
    L.dgs_last_error.restype = ctypes.c_char_p
    L.dgs_workspace_bytes.restype = sz
    L.dgs_workspace_bytes.argtypes = [i32, i32, P(Camera), P(Tuning), i32, i64]
    common = [P(Scene), P(Camera), P(States), P(Tuning), vp, sz]
    L.dgs_count_instances.restype = ctypes.c_int
    L.dgs_count_instances.argtypes = common + [P(i64), vp]
    for name in ("dgs_render", "dgs_render_per_state"):
        f = getattr(L, name)
        f.restype = ctypes.c_int
        f.argtypes = common + [i64, vp, vp, vp]
    L.dgs_render_noalloc.restype = ctypes.c_int
    L.dgs_render_noalloc.argtypes = [P(Scene), P(Camera), P(States), P(Tuning), i64, vp, vp, vp, vp]
    L.dgs_composite_launch.restype = ctypes.c_int
    L.dgs_composite_launch.argtypes = [P(Camera), P(Tuning), i32, P(i32), P(i32), P(i64), P(i64), P(i32)]
    L.dgs_bin.restype = ctypes.c_int
    L.dgs_bin.argtypes = common + [i64, vp]
    L.dgs_composite.restype = ctypes.c_int
    L.dgs_composite.argtypes = common + [i64, vp, vp, vp]
    L.dgs_composite_psnr.restype = ctypes.c_int
    L.dgs_composite_psnr.argtypes = common + [i64, vp, vp, vp]
    L.dgs_composite_stats.restype = ctypes.c_int
    L.dgs_composite_stats.argtypes = common + [i64, vp, vp]
    L.dgs_render_psnr.restype = ctypes.c_int
    L.dgs_render_psnr.argtypes = common + [i64, vp, vp, vp]
    L.dgs_backward.restype = ctypes.c_int
    L.dgs_backward.argtypes = common + [i64, vp, vp, P(SceneGrad), vp]
    L.dgs_check.restype = ctypes.c_int
    L.dgs_check.argtypes = [vp, sz, P(i64), vp]
    L.dgs_workspace_sections.restype = ctypes.c_int
    L.dgs_workspace_sections.argtypes = [i32, i32, P(Camera), P(Tuning), i32, i64, P(WorkspaceView)]
    fp = ctypes.c_float
    L.dgs_utility_workspace_bytes.restype = sz
    L.dgs_utility_workspace_bytes.argtypes = [i32, P(Camera), P(Tuning), i32, i32, i64]
    L.dgs_utility_count.restype = ctypes.c_int
    L.dgs_utility_count.argtypes = common + [i64, vp, vp, i32, vp, sz, P(i64), vp]
    L.dgs_utility.restype = ctypes.c_int
    L.dgs_utility.argtypes = common + [i64, vp, vp, i32, vp, fp, vp, sz, i64, vp, vp]
    L.dgs_utility_check.restype = ctypes.c_int
    L.dgs_utility_check.argtypes = [vp, sz, i64, P(i64), vp]
    L.dgs_distortion_scratch_bytes.restype = sz
    L.dgs_distortion_scratch_bytes.argtypes = [i32, i32, i32]
    L.dgs_distortion.restype = ctypes.c_int
    L.dgs_distortion.argtypes = [vp, i32, i32, i32, vp, fp, vp, sz, vp, vp]
    L.dgs_risk_adjusted.restype = ctypes.c_int
    L.dgs_risk_adjusted.argtypes = [vp, vp, i32, fp, fp, fp, vp, vp]
    L.dgs_sample_states.restype = ctypes.c_int
    L.dgs_sample_states.argtypes = [vp, i32, i32, i32, ctypes.c_uint64, vp, vp]
    L.dgs_objective_scratch_bytes.restype = sz
    L.dgs_objective_scratch_bytes.argtypes = [i32, i32, i32, i32]
    L.dgs_objective.restype = ctypes.c_int
    L.dgs_objective.argtypes = [vp, i32, i32, i32, vp, i32, vp, vp, i32, vp, i32, vp, i32, vp, i32,
                                P(ObjectiveWeights), vp, vp, vp, vp, sz, vp]
    L.dgs_objective_check.restype = ctypes.c_int
    L.dgs_objective_check.argtypes = [vp, sz, vp]
    L.dgs_l1_scratch_bytes.restype = sz
    L.dgs_l1_scratch_bytes.argtypes = [i32, i32, i32]
    L.dgs_l1_loss.restype = ctypes.c_int
    L.dgs_l1_loss.argtypes = [vp, i32, i32, i32, vp, i32, vp, vp, vp, sz, vp]
    L.dgs_l1_loss_grad.restype = ctypes.c_int
    L.dgs_l1_loss_grad.argtypes = [vp, i32, i32, i32, vp, i32, vp, vp, vp, vp]
    L.dgs_probe_copy.restype = ctypes.c_int
    L.dgs_probe_copy.argtypes = [vp, vp, sz, vp]
    L.dgs_probe_valu.restype = ctypes.c_int
    L.dgs_probe_valu.argtypes = [i32, ctypes.c_int64, vp, vp]
    _lib = L
    return L


def check(status: int):
    if status != DGS_OK:
        raise DgsError(status, lib().dgs_last_error().decode())
