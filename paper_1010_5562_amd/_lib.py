"""ctypes declarations of the C ABI in ``include/fcfs.h``.

Loading fails loudly when ``libfcfs.so`` has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfcfs.so")

FCFS_OK = 0
PRECISIONS = {"fp32": 0, "bf16": 1, "fp16": 2, "auto": 3}

STATUS_NAMES = {
    0: "FCFS_OK",
    -1: "FCFS_ERR_INVALID_ARG",
    -2: "FCFS_ERR_NOT_RECTILINEAR",
    -3: "FCFS_ERR_RANGE",
    -4: "FCFS_ERR_UNSUPPORTED",
    -5: "FCFS_ERR_WORKSPACE",
    -6: "FCFS_ERR_DEVICE",
    -7: "FCFS_ERR_NO_MEMORY",
}

# Every symbol the headers under include/ declare (fcfs.h, fcfs_tuning.h).
EXPORTS = (
    "fcfs_create", "fcfs_destroy", "fcfs_set_stream", "fcfs_loops_to_corners",
    "fcfs_workspace_size", "fcfs_forward", "fcfs_forward_noalloc", "fcfs_band_workspace_size", "fcfs_forward_band",
    "fcfs_fft_workspace_size", "fcfs_forward_fft", "fcfs_haar_workspace_size", "fcfs_haar",
    "fcfs_general_workspace_size", "fcfs_forward_general",
    "fcfs_general_band_workspace_size", "fcfs_forward_general_band",
    "fcfs_general_adjoint_workspace_size", "fcfs_adjoint_general", "fcfs_apply_edge_offsets_grid",
    "fcfs_pupil_loss_workspace_size", "fcfs_pupil_loss",
    "fcfs_pupil_step_workspace_size", "fcfs_pupil_step", "fcfs_pupil_step_plan",
    "fcfs_step_plan_launch", "fcfs_step_plan_destroy",
    "fcfs_general_batch_workspace_size", "fcfs_general_batch_plan",
    "fcfs_adjoint", "fcfs_adjoint_band", "fcfs_edge_grad",
    "fcfs_apply_edge_offsets", "fcfs_batch_workspace_size", "fcfs_forward_batch", "fcfs_plan_destroy",
    "fcfs_debug_phases", "fcfs_debug_phases_workspace_size", "fcfs_autotune",
    "fcfs_autotune_batch", "fcfs_batch_choice",
    "fcfs_load_tune", "fcfs_tile_variants", "fcfs_set_tile", "fcfs_forward_plan_info",
    "fcfs_workspace_size_tile", "fcfs_profile_begin", "fcfs_profile_end",
    "fcfs_status_string", "fcfs_last_error",
)


class FcfsClip(ctypes.Structure):
    _fields_ = [
        ("x", ctypes.c_void_p),
        ("y", ctypes.c_void_p),
        ("s", ctypes.c_void_p),
        ("V", ctypes.c_int64),
        ("T", ctypes.c_int32),
        ("K", ctypes.c_int32),
        ("L", ctypes.c_int32),
        ("F", ctypes.c_void_p),
        ("area", ctypes.c_void_p),
    ]


class FcfsGClip(ctypes.Structure):
    _fields_ = [
        ("x", ctypes.c_void_p),
        ("y", ctypes.c_void_p),
        ("s", ctypes.c_void_p),
        ("V", ctypes.c_int64),
        ("Nx", ctypes.c_int32),
        ("Ny", ctypes.c_int32),
        ("frac_bits", ctypes.c_int32),
        ("K", ctypes.c_int32),
        ("L", ctypes.c_int32),
        ("F", ctypes.c_void_p),
        ("area", ctypes.c_void_p),
    ]


class FcfsHaarClip(ctypes.Structure):
    _fields_ = [
        ("x", ctypes.c_void_p),
        ("y", ctypes.c_void_p),
        ("s", ctypes.c_void_p),
        ("poly_off", ctypes.c_void_p),
        ("V", ctypes.c_int64),
        ("M", ctypes.c_int64),
        ("Nx", ctypes.c_int32),
        ("Ny", ctypes.c_int32),
        ("J", ctypes.c_int32),
        ("U", ctypes.c_void_p),
        ("W", ctypes.c_void_p),
        ("stats", ctypes.c_void_p),
    ]


class FcfsError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {detail}")
        self.status = status


_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, c_int = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int
    u32 = ctypes.c_uint32
    sz = ctypes.POINTER(ctypes.c_size_t)
    clip_p = ctypes.POINTER(FcfsClip)
    sig = {
        "fcfs_create": [ctypes.POINTER(P), c_int, P],
        "fcfs_destroy": [P],
        "fcfs_set_stream": [P, P],
        "fcfs_loops_to_corners": [P, P, i64, P, P, P, P, P],
        "fcfs_workspace_size": [clip_p, c_int, c_int, sz],
        "fcfs_workspace_size_tile": [clip_p, c_int, i32, sz],
        "fcfs_forward_plan_info": [clip_p, c_int, ctypes.POINTER(i32), ctypes.POINTER(i64),
                                   ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "fcfs_forward": [P, clip_p, c_int, P, ctypes.c_size_t],
        "fcfs_forward_noalloc": [P, clip_p, c_int],
        "fcfs_band_workspace_size": [clip_p, i32, i32, ctypes.c_double, c_int, sz],
        "fcfs_forward_band": [P, clip_p, i32, i32, ctypes.c_double, c_int, P, ctypes.c_size_t],
        "fcfs_fft_workspace_size": [clip_p, sz],
        "fcfs_forward_fft": [P, clip_p, P, ctypes.c_size_t],
        "fcfs_haar_workspace_size": [ctypes.POINTER(FcfsHaarClip), sz],
        "fcfs_general_workspace_size": [ctypes.POINTER(FcfsGClip), c_int, sz],
        "fcfs_forward_general": [P, ctypes.POINTER(FcfsGClip), c_int, P, ctypes.c_size_t],
        "fcfs_general_band_workspace_size": [ctypes.POINTER(FcfsGClip), i32, i32, ctypes.c_double,
                                             c_int, sz],
        "fcfs_forward_general_band": [P, ctypes.POINTER(FcfsGClip), i32, i32, ctypes.c_double,
                                      c_int, P, ctypes.c_size_t],
        "fcfs_general_adjoint_workspace_size": [ctypes.POINTER(FcfsGClip), c_int, sz],
        "fcfs_adjoint_general": [P, ctypes.POINTER(FcfsGClip), P, i32, i32, ctypes.c_double, P, P,
                                 c_int, P, ctypes.c_size_t],
        "fcfs_apply_edge_offsets_grid": [P, P, P, P, P, P, i64, i32, P, P],
        "fcfs_pupil_loss_workspace_size": [sz],
        "fcfs_pupil_loss": [P, P, P, P, i32, i32, ctypes.c_double, P, P, P, ctypes.c_size_t],
        "fcfs_pupil_step_workspace_size": [i64, i32, i32, i32, i32, i32, ctypes.c_double, c_int,
                                           sz],
        "fcfs_pupil_step": [P, P, P, P, P, P, P, i64, i32, i32, i32, i32, i32, ctypes.c_double,
                            P, P, c_int, P, P, P, P, ctypes.c_size_t],
        "fcfs_pupil_step_plan": [P, P, P, P, P, P, P, i64, i32, i32, i32, i32, i32,
                                 ctypes.c_double, P, P, c_int, P, P, P, P, ctypes.c_size_t,
                                 ctypes.POINTER(P)],
        "fcfs_step_plan_launch": [P, P],
        "fcfs_general_batch_workspace_size": [ctypes.POINTER(FcfsGClip), i32, c_int, sz],
        "fcfs_general_batch_plan": [P, ctypes.POINTER(FcfsGClip), i32, c_int, P, ctypes.c_size_t,
                                    ctypes.POINTER(P)],
        "fcfs_step_plan_destroy": [P],
        "fcfs_haar": [P, ctypes.POINTER(FcfsHaarClip), P, ctypes.c_size_t],
        "fcfs_adjoint": [P, clip_p, P, P, P, c_int, P, ctypes.c_size_t],
        "fcfs_adjoint_band": [P, clip_p, P, i32, i32, ctypes.c_double, P, P, c_int, P,
                              ctypes.c_size_t],
        "fcfs_edge_grad": [P, P, P, P, P, i64, i64, P],
        "fcfs_apply_edge_offsets": [P, P, P, P, P, P, i64, P, P],
        "fcfs_batch_workspace_size": [P, clip_p, i32, c_int, sz],
        "fcfs_forward_batch": [P, clip_p, i32, c_int, P, ctypes.c_size_t, ctypes.POINTER(P)],
        "fcfs_plan_destroy": [P],
        "fcfs_debug_phases": [P, clip_p, i32, i32, i32, P, P, ctypes.c_size_t],
        "fcfs_debug_phases_workspace_size": [i64, i32, sz],
        "fcfs_autotune": [P, ctypes.c_char_p, c_int],
        "fcfs_autotune_batch": [P, clip_p, i32, c_int, c_int],
        "fcfs_batch_choice": [P, c_int, c_int, P, P],
        "fcfs_load_tune": [P, ctypes.c_char_p],
        "fcfs_set_tile": [P, i32],
        "fcfs_profile_begin": [P, u32],
        "fcfs_profile_end": [P, P, P, i32],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = c_int
    lib.fcfs_tile_variants.argtypes = [P, P, i32]
    lib.fcfs_tile_variants.restype = i32
    lib.fcfs_status_string.argtypes = [c_int]
    lib.fcfs_status_string.restype = ctypes.c_char_p
    lib.fcfs_last_error.argtypes = [P]
    lib.fcfs_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(status: int, handle=None) -> None:
    if status != FCFS_OK:
        lib = load()
        detail = lib.fcfs_last_error(handle).decode(errors="replace")
        raise FcfsError(status, detail)
