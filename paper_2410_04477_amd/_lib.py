"""ctypes binding of libvecchia.so (include/vecchia.h).  Argument marshalling
only: every step of the computation runs in the library's HIP kernels.
Importing this module raises if the built library is missing."""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libvecchia.so")

MAX_BUCKETS = 24
MAX_JOINT = 175
ENGINE_MFMA, ENGINE_TILES, ENGINE_MFMA_WG = 0, 1, 2
PLAN_PREDICT = 16
ORDER_MORTON, ORDER_MAXMIN, ORDER_HILBERT, ORDER_KDTREE = 1, 2, 3, 4

OK, EINVAL, ENOMEM, EHIP, EUNSUPPORTED = 0, -1, -2, -3, -4
NOALLOC_MAX_ITEMS = 1 << 20
FP64, FP32_BULK = 0, 1


class Theta(ctypes.Structure):
    _fields_ = [("sigma2", ctypes.c_double), ("range", ctypes.c_double), ("nugget", ctypes.c_double),
                ("nu", ctypes.c_double), ("aniso", ctypes.c_double * 3)]


class Plan(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("bc", ctypes.c_int64), ("max_theta", ctypes.c_int32),
                ("nbuckets", ctypes.c_int32), ("pmax", ctypes.c_int32), ("lmax", ctypes.c_int32),
                ("mmax", ctypes.c_int32), ("bucket_cfg", ctypes.c_int32 * MAX_BUCKETS),
                ("bucket_off", ctypes.c_int64 * (MAX_BUCKETS + 1)), ("lsum", ctypes.c_int64),
                ("flops_la", ctypes.c_double), ("cov_entries", ctypes.c_double),
                ("ws", ctypes.c_void_p), ("ws_bytes", ctypes.c_size_t),
                ("off_sched", ctypes.c_size_t), ("off_partial", ctypes.c_size_t), ("off_flag", ctypes.c_size_t),
                ("off_list", ctypes.c_size_t), ("off_count", ctypes.c_size_t), ("off_chunk", ctypes.c_size_t),
                ("off_grad", ctypes.c_size_t), ("timing", ctypes.c_void_p), ("engine", ctypes.c_int32),
                ("nlarge", ctypes.c_int64), ("large_slots", ctypes.c_int32), ("large_slot_elems", ctypes.c_int64),
                ("aux_ws_bytes", ctypes.c_size_t), ("aux_ws", ctypes.c_void_p),
                ("bucket_lmax", ctypes.c_int32 * MAX_BUCKETS), ("lds_bytes", ctypes.c_int32),
                ("bucket_main", ctypes.c_int32), ("exec", ctypes.c_void_p), ("kind", ctypes.c_int32)]


class VecchiaError(RuntimeError):
    pass


P = ctypes.c_void_p
I32, I64, SZ, D = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_double

# name -> (restype, argtypes); the list mirrors include/vecchia.h
SIGNATURES = {
    "vecchia_version": (ctypes.c_int, []),
    "vecchia_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "vecchia_blocks_workspace_size": (SZ, [I64, I64, I32]),
    "vecchia_blocks": (ctypes.c_int, [P, I64, I32, P, P, P, I64, I32, P, P, P, P, P, SZ, P]),
    "vecchia_neighbors_workspace_size": (SZ, [I64, I64, I32, I32]),
    "vecchia_neighbors": (ctypes.c_int, [P, I64, I32, P, P, I64, I32, P, P, I64, P, SZ, P]),
    "vecchia_plan_workspace_size": (SZ, [I64, I32]),
    "vecchia_plan_init": (ctypes.c_int, [P, P, P, I64, I64, I32, I32, P, SZ, P]),
    "vecchia_loglik": (ctypes.c_int, [P, P, P, I32, P, P, P, P, I32, I32, P, P, P, P]),
    "vecchia_loglik_noalloc": (ctypes.c_int, [P, P, P, I32, P, P, P, P, I32, I32, P, P, P, P]),
    "vecchia_noalloc_scratch_bytes": (SZ, []),
    "vecchia_permute": (ctypes.c_int, [P, I64, I32, P, P, P]),
    "vecchia_loglik_grad": (ctypes.c_int, [P, P, P, I32, P, P, P, P, I32, I32, P, P, P, P, P, P]),
    "vecchia_loglik_dnu": (ctypes.c_int, [P, P, P, I32, P, P, P, P, I32, ctypes.c_double, P, P, P]),
    "vecchia_loglik_grad_nu": (ctypes.c_int, [P, P, P, I32, P, P, P, P, I32, I32, P, P, P, P, P, P, P, P]),
    "vecchia_simulate_workspace_size": (SZ, [I64, I64, I32]),
    "vecchia_simulate": (ctypes.c_int, [P, I64, I32, P, P, P, I32, P, P, P, SZ, P]),
    "vecchia_variogram_workspace_size": (SZ, [I32, I32, I32]),
    "vecchia_variogram": (ctypes.c_int, [P, I64, P, I64, I32, I32, I32, D, P, I32, P, P, I32, P, SZ, P]),
    "vecchia_gemm": (ctypes.c_int, [P, P, P, P, P, P, I32, I32, I32, I32, I32, I32, I32, I32, I32, I32, I32, P]),
    "vecchia_mse": (ctypes.c_int, [P, P, I32, P, P, I32, P]),
    "vecchia_colsum": (ctypes.c_int, [P, I32, I32, I32, P, P]),
    "vecchia_adam": (ctypes.c_int, [P, P, P, P, I64, D, D, D, D, I64, P]),
    "vecchia_tile_config": (ctypes.c_int, [I32, I32, P, P]),
    "vecchia_plan_attach_aux": (ctypes.c_int, [P, P, SZ]),
    "vecchia_plan_destroy": (ctypes.c_int, [P]),
    "vecchia_plan_set_timing": (ctypes.c_int, [P, ctypes.c_int]),
    "vecchia_plan_timing": (ctypes.c_int, [P, P, P, ctypes.c_int]),
    "vecchia_pred_neighbors_workspace_size": (SZ, [I64, I64, I64, I32, I32]),
    "vecchia_pred_neighbors": (ctypes.c_int, [P, I64, P, I64, I32, P, P, I64, I32, P, P, I64, P, SZ, P]),
    "vecchia_predict": (ctypes.c_int, [P, P, P, P, I32, P, P, P, P, P, P, P, I32, P]),
    "vecchia_reorder_blocks_workspace_size": (SZ, [I64, I64, I32]),
    "vecchia_reorder_blocks": (ctypes.c_int, [P, I64, I32, P, P, I64, I32, P, P, P, P, SZ, P]),
    "vecchia_condsim_workspace_size": (SZ, [I64]),
    "vecchia_condsim": (ctypes.c_int, [P, P, I64, P, I32, P, P, P, P, P, P, P, SZ, P]),
    "vecchia_plan_layout": (I32, [P, I32]),
    "vecchia_plan_class_kernel": (ctypes.c_int, [P, I32, I32, I32, ctypes.c_char_p, I32]),
}

_lib = None


def plan_layout_mismatch(L: ctypes.CDLL, cls=Plan):
    """None if the ctypes mirror `cls` has the library's vecchia_plan layout
    (size and every field offset, in order), else a description of the first
    difference."""
    k = L.vecchia_plan_layout(None, 0)
    buf = (ctypes.c_int64 * k)()
    L.vecchia_plan_layout(buf, k)
    lib_layout = list(buf)
    mine = [ctypes.sizeof(cls)] + [getattr(cls, f[0]).offset for f in cls._fields_]
    if lib_layout == mine:
        return None
    names = ["sizeof"] + [f[0] for f in cls._fields_]
    for i in range(max(len(mine), len(lib_layout))):
        a = lib_layout[i] if i < len(lib_layout) else None
        b = mine[i] if i < len(mine) else None
        if a != b:
            what = names[i] if i < len(names) else f"entry {i}"
            return f"vecchia_plan {what}: library {a}, binding {b}"
    return "vecchia_plan layout differs"


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise VecchiaError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run `python -m paper_2410_04477_amd.build`)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name, None)
            if f is None:
                continue
            f.restype = res
            f.argtypes = args
        bad = plan_layout_mismatch(L)
        if bad:
            raise VecchiaError(f"binding and library disagree on the plan layout ({bad}): rebuild the library")
        _lib = L
    return _lib


def check(status: int, what: str) -> None:
    if status != OK:
        msg = lib().vecchia_status_string(status).decode()
        raise VecchiaError(f"{what} failed: {msg} ({status})")
