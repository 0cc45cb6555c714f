"""ctypes declarations of the C ABI in ``include/pic.h`` (argument marshalling only).

The shared library is loaded after ``torch`` so that both use the one HIP
runtime torch brings (same SONAME); device pointers of torch tensors are then
valid in the library.  A missing library raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpic.so")

PIC_OK, PIC_EINVAL, PIC_ENOMEM, PIC_EDEVICE, PIC_ESTATE, PIC_ECAPACITY, PIC_ENONFINITE = 0, -1, -2, -3, -4, -5, -6
PIC_EULER, PIC_RK2, PIC_RK4 = 1, 2, 4
PIC_F64, PIC_F32 = 0, 1
PIC_INTERP_CELL_AVERAGE, PIC_INTERP_LINEAR_LS, PIC_INTERP_GEOMETRIC_AVERAGE, PIC_INTERP_HARMONIC_AVERAGE = 0, 1, 2, 3
PIC_INTERP_NEAREST, PIC_INTERP_INV_DISTANCE, PIC_INTERP_SHAPE_WEIGHTED = 4, 5, 6
PIC_PROP_GIVEN, PIC_PROP_INITIAL_POSITION = 0, 1
PIC_LOST = 0xFFFFFFFF

STATUS_NAMES = {0: "PIC_OK", -1: "PIC_EINVAL", -2: "PIC_ENOMEM", -3: "PIC_EDEVICE", -4: "PIC_ESTATE",
                -5: "PIC_ECAPACITY", -6: "PIC_ENONFINITE"}

# every exported function of include/pic.h (checked by the CPU tests)
EXPORTS = [
    "pic_create", "pic_set_stream", "pic_destroy", "pic_last_error",
    "pic_mesh_uniform", "pic_mesh_displace", "pic_mesh_octree", "pic_mesh_info", "pic_q2_nodes",
    "pic_set_velocity", "pic_set_velocity_end", "pic_shift_velocity", "pic_set_field_time", "pic_field_time",
    "pic_scratch_bytes", "pic_bind_store", "pic_current_buffer", "pic_set_tile",
    "pic_seed_reference", "pic_seed_per_cell", "pic_seed_positions", "pic_set_property_odes", "pic_advance", "pic_population",
    "pic_interpolate", "pic_interpolate_points", "pic_seed_mh", "pic_seed_mh_static", "pic_transfer", "pic_set_launch_graphs",
    "pic_adjoint_workspace_bytes", "pic_advance_checkpointed", "pic_adjoint",
    "pic_stats_read", "pic_stats_reset", "pic_profile_enable", "pic_profile_read",
    "pic_batch_create", "pic_batch_advance", "pic_batch_set_schedule", "pic_batch_tune", "pic_batch_destroy",
    "pic_batch_tune_cache_write", "pic_batch_tune_cache_apply",
    "pic_batch_last_error",
]


class PicStore(C.Structure):
    _fields_ = [("capacity", C.c_int64),
                ("x", C.c_void_p * 2), ("xr", C.c_void_p * 2), ("cell", C.c_void_p * 2), ("id", C.c_void_p * 2),
                ("prop", C.c_void_p * 2), ("cell_start", C.c_void_p * 2),
                ("n_prop", C.c_int32), ("prop_prec", C.c_int32),
                ("scratch", C.c_void_p), ("scratch_bytes", C.c_int64)]


class PicStats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in ("live", "lost", "moved", "near_face", "first_try", "fallback",
                                         "newton_fail", "added", "deleted", "steps", "particle_steps",
                                         "searches", "searched")]


class PicError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lock = threading.Lock()
_lib = None


def load(path: str | None = None):
    """Load libpic.so (after torch); raise if it is not built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        import torch  # noqa: F401  (binds the HIP runtime torch ships before the library loads)
        p = path or LIB_PATH
        if not os.path.exists(p):
            raise RuntimeError(f"{p} is not built; run __graft_entry__.build() or "
                               "python paper_1612_03369_amd/build.py")
        L = C.CDLL(p, mode=C.RTLD_GLOBAL)
        P, I32, I64, D, U64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_uint64
        S = C.c_int
        sig = {
            "pic_create": (S, [C.POINTER(P), C.c_int, P]),
            "pic_set_stream": (S, [P, P]),
            "pic_destroy": (None, [P]),
            "pic_last_error": (C.c_char_p, [P]),
            "pic_mesh_uniform": (S, [P, C.c_int, P, P, P]),
            "pic_mesh_displace": (S, [P, P]),
            "pic_mesh_octree": (S, [P, P, P, C.c_int, I64, P, P]),
            "pic_mesh_info": (S, [P, P, P, P]),
            "pic_q2_nodes": (S, [P, P, P]),
            "pic_set_velocity": (S, [P, P, C.c_int]),
            "pic_scratch_bytes": (S, [P, I64, P]),
            "pic_bind_store": (S, [P, C.POINTER(PicStore)]),
            "pic_current_buffer": (S, [P, P]),
            "pic_set_tile": (S, [P, I32]),
            "pic_seed_reference": (S, [P, P, P, P, I64, I32, P]),
            "pic_seed_per_cell": (S, [P, P, C.c_uint64, C.c_uint32, I32, P]),
            "pic_seed_positions": (S, [P, P, P, I64, I32, P]),
            "pic_advance": (S, [P, D, I32, I32, I32]),
            "pic_set_property_odes": (S, [P, I32, I32, C.c_double, C.c_double]),
            "pic_set_velocity_end": (S, [P, P, I32, C.c_double]),
            "pic_interpolate_points": (S, [P, I32, P, I32, P, P]),
            "pic_seed_mh": (S, [P, P, P, I32, C.c_uint64, C.c_uint32, P]),
            "pic_seed_mh_static": (S, [P, P, P, I32, C.c_uint64, C.c_uint32, P]),
            "pic_set_launch_graphs": (S, [P, I32]),
            "pic_transfer": (S, [P, P]),
            "pic_shift_velocity": (S, [P, P, I32, C.c_double]),
            "pic_set_field_time": (S, [P, C.c_double]),
            "pic_field_time": (S, [P, P]),
            "pic_population": (S, [P, I32, I32, U64, U64]),
            "pic_interpolate": (S, [P, I32, P, P, P]),
            "pic_adjoint_workspace_bytes": (S, [P, I32, I32, P]),
            "pic_advance_checkpointed": (S, [P, D, I32, I32, I32, P]),
            "pic_adjoint": (S, [P, P, P, P]),
            "pic_stats_read": (S, [P, C.POINTER(PicStats)]),
            "pic_stats_reset": (S, [P]),
            "pic_profile_enable": (S, [P, I32]),
            "pic_profile_read": (S, [P, C.c_char_p, P, P]),
            "pic_batch_create": (S, [C.POINTER(P), I32, P, P, P]),
            "pic_batch_advance": (S, [P, P, P, I32]),
            "pic_batch_set_schedule": (S, [P, P]),
            "pic_batch_tune": (S, [P, P, P, I32, P, P]),
            "pic_batch_tune_cache_write": (S, [P, P, C.c_char_p, C.c_int64, P]),
            "pic_batch_tune_cache_apply": (S, [P, P, C.c_char_p, P]),
            "pic_batch_destroy": (None, [P]),
            "pic_batch_last_error": (C.c_char_p, [P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
        return L


def check(status: int, ctx=None, batch=None):
    if status == PIC_OK:
        return
    L = load()
    if batch is not None:
        msg = L.pic_batch_last_error(batch)
    else:
        msg = L.pic_last_error(ctx) if ctx is not None else b""
    raise PicError(status, (msg or b"").decode())
