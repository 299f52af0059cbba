"""ctypes wrapper and gcc build of the plain-C oracle (csrc/bv_oracle.c)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "bv_oracle.c")
_LIB = os.path.join(_HERE, "_build", "libbv_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no fused multiply-add, OpenMP)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        for name in ("bvo_loglik", "bvo_grad"):
            f = getattr(L, name)
            f.restype = ctypes.c_int64
            f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                          ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]
        for name in ("bvo_loglik_sel", "bvo_grad_sel"):
            f = getattr(L, name)
            f.restype = ctypes.c_int64
            f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                          ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int32]
        f = L.bvo_simulate
        f.restype = ctypes.c_int64
        f.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        _lib = L
    return _lib


def _theta7(theta):
    if theta.nu not in (0.5, 1.5, 2.5):
        raise ValueError("C oracle supports nu in {0.5, 1.5, 2.5}")
    a = tuple(theta.aniso) + (1.0,) * (3 - len(theta.aniso))
    return np.array([theta.sigma2, theta.beta, theta.nugget, theta.nu, a[0], a[1], a[2]], dtype=np.float64)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def block_terms(locs_perm, y_perm, block_ptr, nbr_ptr, nbr_idx, theta, nthreads: int = 0):
    """Per-block terms l_i = log N(y_J) - log N(y_N) in FP64; NaN marks a non-PD block."""
    locs = _c(locs_perm, np.float64)
    y = _c(y_perm, np.float64)
    bp = _c(block_ptr, np.int64)
    npt = _c(nbr_ptr, np.int64)
    ni = _c(nbr_idx, np.int64) if len(nbr_idx) else np.zeros(1, np.int64)
    th = _theta7(theta)
    bc = bp.size - 1
    out = np.empty(bc, np.float64)
    lib().bvo_loglik(locs.ctypes.data, y.ctypes.data, locs.shape[0], locs.shape[1], bp.ctypes.data, bc,
                     npt.ctypes.data, ni.ctypes.data, th.ctypes.data, out.ctypes.data, nthreads)
    return out


def loglik(locs_perm, y_perm, block_ptr, nbr_ptr, nbr_idx, theta, nthreads: int = 0) -> float:
    t = block_terms(locs_perm, y_perm, block_ptr, nbr_ptr, nbr_idx, theta, nthreads)
    acc = 0.0
    for v in t:  # block order
        acc += float(v)
    return acc


def grad_terms(locs_perm, y_perm, block_ptr, nbr_ptr, nbr_idx, theta, nthreads: int = 0):
    """Per-block gradient rows (bc x 3) w.r.t. (sigma2, beta, nugget)."""
    locs = _c(locs_perm, np.float64)
    y = _c(y_perm, np.float64)
    bp = _c(block_ptr, np.int64)
    npt = _c(nbr_ptr, np.int64)
    ni = _c(nbr_idx, np.int64) if len(nbr_idx) else np.zeros(1, np.int64)
    th = _theta7(theta)
    bc = bp.size - 1
    out = np.empty((bc, 3), np.float64)
    lib().bvo_grad(locs.ctypes.data, y.ctypes.data, locs.shape[0], locs.shape[1], bp.ctypes.data, bc,
                   npt.ctypes.data, ni.ctypes.data, th.ctypes.data, out.ctypes.data, nthreads)
    return out


def grad(locs_perm, y_perm, block_ptr, nbr_ptr, nbr_idx, theta, nthreads: int = 0) -> np.ndarray:
    g = grad_terms(locs_perm, y_perm, block_ptr, nbr_ptr, nbr_idx, theta, nthreads)
    acc = np.zeros(3)
    for row in g:
        acc = acc + row
    return acc


def simulate(locs_perm, block_ptr, nbr_ptr, nbr_idx, theta, z):
    """Draw y (block order) from the block Vecchia density, blocks in order.
    With unit blocks and nearest-earlier-point neighbours this is the
    sequential Vecchia simulator."""
    locs = _c(locs_perm, np.float64)
    bp = _c(block_ptr, np.int64)
    npt = _c(nbr_ptr, np.int64)
    ni = _c(nbr_idx, np.int64) if len(nbr_idx) else np.zeros(1, np.int64)
    zz = _c(z, np.float64)
    y = np.zeros(locs.shape[0])
    bad = lib().bvo_simulate(locs.ctypes.data, locs.shape[0], locs.shape[1], bp.ctypes.data, bp.size - 1,
                             npt.ctypes.data, ni.ctypes.data, _theta7(theta).ctypes.data, zz.ctypes.data,
                             y.ctypes.data)
    if bad:
        raise ValueError(f"{bad} blocks not positive definite in simulation")
    return y


def selected_terms(locs_perm, y_perm, block_ptr, nbr_ptr, nbr_idx, theta, sel, with_grad=False, nthreads=0):
    """Per-block terms (and gradient rows) of the blocks listed in sel only."""
    locs = _c(locs_perm, np.float64)
    y = _c(y_perm, np.float64)
    bp = _c(block_ptr, np.int64)
    npt = _c(nbr_ptr, np.int64)
    ni = _c(nbr_idx, np.int64) if len(nbr_idx) else np.zeros(1, np.int64)
    sl = _c(sel, np.int64)
    th = _theta7(theta)
    out = np.empty(sl.size)
    lib().bvo_loglik_sel(locs.ctypes.data, y.ctypes.data, locs.shape[0], locs.shape[1], bp.ctypes.data,
                         bp.size - 1, npt.ctypes.data, ni.ctypes.data, th.ctypes.data, sl.ctypes.data, sl.size,
                         out.ctypes.data, nthreads)
    if not with_grad:
        return out
    g = np.empty((sl.size, 3))
    lib().bvo_grad_sel(locs.ctypes.data, y.ctypes.data, locs.shape[0], locs.shape[1], bp.ctypes.data,
                       bp.size - 1, npt.ctypes.data, ni.ctypes.data, th.ctypes.data, sl.ctypes.data, sl.size,
                       g.ctypes.data, nthreads)
    return out, g
