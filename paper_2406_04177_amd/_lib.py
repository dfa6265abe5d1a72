"""ctypes binding of libvgsim.so (declared in include/vgsim.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  The library must have been built (``python -m
paper_2406_04177_amd.build``); there is no fallback, a missing library is an
error.
"""
from __future__ import annotations

import ctypes
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("VGSIM_LIB") or os.path.join(_HERE, "libvgsim.so")

VG_OK, VG_EINVAL, VG_EUNSTABLE, VG_ENOCONV, VG_ENONFINITE, VG_EHIP, VG_ESTATE = 0, -1, -2, -3, -4, -5, -6
VG_F32, VG_F64, VG_F32C = 0, 1, 2
VG_ORDER_TD, VG_ORDER_DT = 0, 1
VG_FORCE = 1
VG_FEAT_CG, VG_FEAT_ADJ, VG_FEAT_BAND, VG_FEAT_MG = 1, 2, 4, 8
VG_PRECOND_JACOBI, VG_PRECOND_MG = 0, 1
VG_MG_MAX_LEVELS = 12
VG_NPOOL, VG_NREG, VG_NGRAD = 5, 8, 20
VG_KERNEL_AUTO, VG_KERNEL_TABLE, VG_KERNEL_RANK, VG_KERNEL_OFFSET, VG_KERNEL_RELATIVE, VG_KERNEL_BAND = 0, 1, 2, 3, 4, 5
VG_ADJ_SKIP_STATIC_D, VG_ADJ_TAPE_DOM = 1, 2
VG_PNGM_NOALLOC_MAX_Q = 65536
VG_LAUNCH_GRAPHS_AUTO, VG_LAUNCH_GRAPHS_ON, VG_LAUNCH_GRAPHS_OFF = 0, 1, 2

EXPORTS = ("vg_strerror", "vg_last_error", "vg_version", "vg_rank_bytes", "vg_count_pores",
           "vg_build_graph", "vg_lookup", "vg_region_codes", "vg_range_sums",
           "vg_brick_stats", "vg_pngm_partition_bytes", "vg_pngm_partition", "vg_pngm_loss_grad", "vg_pngm_step", "vg_pngm_implicit_step",
           "vg_pngm_implicit_step_noalloc", "vg_sign_update", "vg_create", "vg_destroy",
           "vg_set_kernel", "vg_get_kernel", "vg_set_launch_options", "vg_set_adjoint_options", "vg_set_params", "vg_set_regions", "vg_alt_elems", "vg_workspace_bytes", "vg_init_state",
           "vg_step_explicit", "vg_step_subcycled", "vg_solve_implicit_step", "vg_set_preconditioner",
           "vg_mg_levels", "vg_precondition", "vg_mass_totals", "vg_record", "vg_adjoint",
           "vg_seed_lambda", "vg_load_state", "vg_store_state", "vg_step_record", "vg_tape_rows")


class VgError(RuntimeError):
    def __init__(self, code: int, where: str, text: str):
        super().__init__("%s failed: %s (%d): %s" % (where, _strerror(code), code, text))
        self.code = code


class VgParams(ctypes.Structure):
    _fields_ = [("D", ctypes.c_double * 5), ("h", ctypes.c_double), ("v_dom", ctypes.c_double),
                ("k_dom", ctypes.c_double), ("rho", ctypes.c_double), ("mu", ctypes.c_double),
                ("beta", ctypes.c_double), ("v_som", ctypes.c_double), ("v_p4", ctypes.c_double),
                ("mort_to_p4", ctypes.c_int32), ("step_order", ctypes.c_int32), ("sequential", ctypes.c_int32)]


class VgDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nseg", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("seg_off", ctypes.c_void_p), ("nbr_d", ctypes.c_void_p), ("rcode_d", ctypes.c_void_p),
                ("mobile_all", ctypes.c_int32), ("features", ctypes.c_int32),
                ("rank_d", ctypes.c_void_p), ("vox_d", ctypes.c_void_p), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("brick", ctypes.c_int32), ("periodic", ctypes.c_uint32)]


_lock = threading.Lock()
_lib = None


def load():
    """Load libvgsim.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libvgsim.so is not built (%s); run `python -m paper_2406_04177_amd.build`"
                               % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        P, I, I64, D, U = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_uint
        S = ctypes.c_size_t
        sig = {
            "vg_strerror": (ctypes.c_char_p, [I]),
            "vg_last_error": (ctypes.c_char_p, []),
            "vg_version": (I, []),
            "vg_rank_bytes": (I, [I, I, I, I, ctypes.POINTER(S)]),
            "vg_count_pores": (I, [P, I, I, I, I, P, ctypes.POINTER(I64), P]),
            "vg_build_graph": (I, [P, I, I, I, I, U, ctypes.c_int32, I64, I64, P, P, P]),
            "vg_lookup": (I, [P, I, I, I, I, P, I64, ctypes.c_int32, P, P]),
            "vg_region_codes": (I, [P, I64, I, I, I, U, P, P]),
            "vg_range_sums": (I, [P, I, I64, P, I64, P, P]),
            "vg_brick_stats": (I, [P, P, I64, I, I, I, I, P, P, P]),
            "vg_pngm_partition_bytes": (I, [I, I, I, I, ctypes.POINTER(S), ctypes.POINTER(I64), ctypes.POINTER(I64)]),
            "vg_pngm_partition": (I, [P, P, I64, I, I, I, I, P, S, P, P, P, P, P, P, P,
                                      ctypes.POINTER(I64), ctypes.POINTER(I64), P]),
            "vg_pngm_loss_grad": (I, [P, P, I64, I64, P, P, P, P, D, I, P, P, P, P]),
            "vg_pngm_step": (I, [P, P, I64, P, P, P, P, D, P]),
            "vg_pngm_implicit_step": (I, [P, P, I64, P, P, P, P, D, D, I, P, P, P, P]),
            "vg_pngm_implicit_step_noalloc": (I, [P, P, I64, P, P, P, P, D, D, I, P, P, P]),
            "vg_sign_update": (I, [P, P, I64, D, P, P, P, P]),
            "vg_create": (I, [ctypes.POINTER(VgDesc), ctypes.POINTER(P)]),
            "vg_destroy": (I, [P]),
            "vg_set_kernel": (I, [P, I]),
            "vg_get_kernel": (I, [P, ctypes.POINTER(I)]),
            "vg_set_launch_options": (I, [P, U]),
            "vg_set_adjoint_options": (I, [P, ctypes.c_uint]),
            "vg_set_params": (I, [P, ctypes.POINTER(VgParams)]),
            "vg_set_regions": (I, [P, ctypes.POINTER(D)]),
            "vg_alt_elems": (I, [P, ctypes.POINTER(I64)]),
            "vg_workspace_bytes": (I, [P, ctypes.POINTER(S)]),
            "vg_init_state": (I, [P, P, P, P, S, P]),
            "vg_step_explicit": (I, [P, I64, D, I64, P, U, P]),
            "vg_step_subcycled": (I, [P, I64, D, D, U, P]),
            "vg_solve_implicit_step": (I, [P, D, D, I, P, P, P]),
            "vg_set_preconditioner": (I, [P, I]),
            "vg_mg_levels": (I, [P, ctypes.POINTER(I), P]),
            "vg_precondition": (I, [P, D, P, P, P]),
            "vg_mass_totals": (I, [P, P, P]),
            "vg_record": (I, [P, I64, D, P, P]),
            "vg_step_record": (I, [P, I64, D, P, P, U, P]),
            "vg_tape_rows": (I, [P]),
            "vg_adjoint": (I, [P, I64, D, P, P, P, P, P]),
            "vg_seed_lambda": (I, [P, P, P, I, P]),
            "vg_load_state": (I, [P, P, I, P]),
            "vg_store_state": (I, [P, P, I, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
        return L


def _strerror(code: int) -> str:
    try:
        return load().vg_strerror(code).decode()
    except Exception:  # pragma: no cover - only when the library itself is missing
        return "error"


def check(rc: int, where: str) -> int:
    """Raise VgError for a negative status."""
    if rc < 0:
        raise VgError(rc, where, load().vg_last_error().decode())
    return rc


def stream_ptr(stream=None) -> int:
    """hipStream_t of a torch stream (default: the current stream) as an int."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream
