"""ctypes declarations of libpbf's C ABI (include/pbf.h).

Argument marshalling only: every step of the solver runs in the HIP
kernels of libpbf.so.  Loading fails loudly when the library is not built.
"""
from __future__ import annotations

import ctypes
from pathlib import Path

LIB_PATH = Path(__file__).resolve().parent / "libpbf.so"

PBF_OK = 0
PBF_ERR_INVALID_ARG = -1
PBF_ERR_NONFINITE = -2
PBF_ERR_OUT_OF_MEMORY = -3
PBF_ERR_DEVICE = -4
PBF_ERR_CAPACITY = -5

PBF_MAX_ITERS = 32
PBF_MAX_CELL = 4096
PBF_DEFAULT_NEIGHBOURS = 96
PBF_MAX_SCENES = 65535
PBF_STATIC_SCRATCH_BYTES = 64 << 20

PBF_LOD_UNIFORM = 0
PBF_LOD_EXPLICIT = 1
PBF_LOD_DTC = 2
PBF_LOD_DTVS = 3
PBF_MAX_SPLAT = 16
PBF_MAX_IMAGE = 8192
PBF_MAX_CAMERAS = 4
PBF_FLAG_UNILATERAL = 1

PBF_MAX_OBSTACLES = 4
PBF_OBSTACLE_SPHERE = 1
PBF_OBSTACLE_CONE = 2
PBF_OBSTACLE_BOX = 3

c_i32, c_i64, c_u32, c_f32, c_vp = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                    ctypes.c_float, ctypes.c_void_p)


class PbfParams(ctypes.Structure):
    _fields_ = [("n", c_i32), ("n_min", c_i32), ("n_max", c_i32), ("grid_dims", c_i32 * 3),
                ("box_lo", c_f32 * 3), ("box_hi", c_f32 * 3), ("h", c_f32), ("rho0", c_f32),
                ("mass", c_f32), ("eps", c_f32), ("dt", c_f32), ("gravity", c_f32 * 3),
                ("max_neighbours", c_i32), ("flags", c_u32)]


class PbfLodDesc(ctypes.Structure):
    _fields_ = [("mode", c_i32), ("levels", c_vp), ("levels_on_device", c_i32),
                ("camera", c_f32 * 3), ("d_near", c_f32), ("d_far", c_f32),
                ("forward", c_f32 * 3), ("up", c_f32 * 3), ("focal", c_f32),
                ("width", c_i32), ("height", c_i32), ("splat", c_f32),
                ("n_extra_cameras", c_i32), ("extra_camera", (c_f32 * 3) * (PBF_MAX_CAMERAS - 1)),
                ("extra_range", (c_f32 * 2) * (PBF_MAX_CAMERAS - 1)), ("auto_range", c_i32)]


class PbfObstacle(ctypes.Structure):
    _fields_ = [("kind", c_i32), ("centre", c_f32 * 3), ("a", c_f32 * 3)]


class PbfContactDesc(ctypes.Structure):
    _fields_ = [("count", c_i32), ("obstacles", PbfObstacle * PBF_MAX_OBSTACLES),
                ("stab_iters", c_i32), ("stab_set", c_i32)]


class PbfStepStats(ctypes.Structure):
    _fields_ = [("n_iters", c_i32), ("active", c_i64 * PBF_MAX_ITERS),
                ("particle_iterations", c_i64), ("neighbour_pairs", c_i64),
                ("max_neighbours", c_i32), ("total_particle_iterations", c_i64),
                ("total_steps", c_i64), ("max_stage", c_i32), ("tiles_unstaged", c_i32)]


P = ctypes.POINTER
CTX = c_vp

# name -> (restype, argtypes); every extern "C" function of include/pbf.h
SIGNATURES = {
    "pbf_create": (c_i32, [P(PbfParams), c_vp, c_vp, c_i32, c_vp, P(CTX)]),
    "pbf_set_lod": (c_i32, [CTX, P(PbfLodDesc)]),
    "pbf_step": (c_i32, [CTX, c_i32]),
    "pbf_read_positions": (c_i32, [CTX, c_vp, c_i32]),
    "pbf_read_velocities": (c_i32, [CTX, c_vp, c_i32]),
    "pbf_sync": (c_i32, [CTX]),
    "pbf_destroy": (None, [CTX]),
    "pbf_last_error": (ctypes.c_char_p, [CTX]),
    "pbf_status_string": (ctypes.c_char_p, [c_i32]),
    "pbf_batch_create": (c_i32, [c_i32, P(PbfParams), c_vp, c_vp, c_i32, c_vp, P(CTX)]),
    "pbf_batch_set_lod": (c_i32, [CTX, c_i32, P(PbfLodDesc)]),
    "pbf_batch_set_obstacles": (c_i32, [CTX, c_i32, P(PbfContactDesc)]),
    "pbf_batch_set_cohesion": (c_i32, [CTX, c_i32, c_f32]),
    "pbf_batch_read_positions": (c_i32, [CTX, c_i32, c_vp, c_i32]),
    "pbf_get_counts": (c_i32, [CTX, P(c_i32), P(c_i64)]),
    "pbf_set_memory_limit": (c_i32, [c_i64]),
    "pbf_device_bytes": (c_i64, []),
    "pbf_set_graph": (c_i32, [CTX, c_i32]),
    "pbf_kernel_count": (c_i32, []),
    "pbf_kernel_name": (ctypes.c_char_p, [c_i32]),
    "pbf_set_block_size": (c_i32, [CTX, c_i32, c_i32]),
    "pbf_profile_enable": (c_i32, [CTX, c_i32]),
    "pbf_profile_read": (c_i32, [CTX, c_vp, c_vp, c_i32]),
    "pbf_stats": (c_i32, [CTX, P(PbfStepStats)]),
    "pbf_debug_keys": (c_i32, [CTX, c_vp]),
    "pbf_debug_permutation": (c_i32, [CTX, c_vp]),
    "pbf_debug_neighbours": (c_i32, [CTX, c_vp, c_vp, c_i64, P(c_i64)]),
    "pbf_debug_lambda": (c_i32, [CTX, c_vp]),
    "pbf_debug_levels": (c_i32, [CTX, c_vp]),
    "pbf_debug_contacts": (c_i32, [CTX, c_vp]),
    "pbf_debug_poison": (c_i32, [CTX, c_i32]),
    "pbf_get_state": (c_i32, [CTX, c_vp, c_vp, P(c_i64)]),
    "pbf_set_state": (c_i32, [CTX, c_vp, c_vp, c_i64]),
    "pbf_density": (c_i32, [CTX, c_vp, c_vp, c_i32]),
    "pbf_density_noalloc": (c_i32, [CTX, c_vp, c_vp, c_i32]),
    "pbf_rollout_forward": (c_i32, [CTX, c_i32, c_i32]),
    "pbf_rollout_backward": (c_i32, [CTX, c_vp, c_vp, c_vp, c_vp, c_i32]),
}

_lib = None


def load():
    """Load libpbf.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                              "(or python -m paper_1608_04721_amd.build)")
        lib = ctypes.CDLL(str(LIB_PATH))
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib
