"""Python face of the block Vecchia library.  PyTorch supplies device memory
and the current HIP stream; all computation happens in libvecchia.so."""
from __future__ import annotations

import ctypes
from typing import Iterable, Optional, Sequence

import torch

from . import _lib as L

PRECISIONS = {"fp64": L.FP64, "fp32": L.FP32_BULK, "fp32_bulk": L.FP32_BULK, "fp32_force_refactor": 2}


def _stream(device: Optional[torch.device] = None) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _p(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev_check(*ts: torch.Tensor) -> torch.device:
    dev = None
    for t in ts:
        if t is None:
            continue
        if not t.is_cuda:
            raise ValueError("tensors must live on the HIP device")
        if not t.is_contiguous():
            raise ValueError("tensors must be contiguous")
        dev = t.device if dev is None else dev
    return dev


def make_theta(th) -> L.Theta:
    """Accepts an object with sigma2/beta(or range)/nugget/nu/aniso, or a tuple
    (sigma2, range, nugget, nu[, aniso])."""
    if isinstance(th, L.Theta):
        return th
    if isinstance(th, (tuple, list)):
        s2, rg, nug, nu = th[:4]
        an = th[4] if len(th) > 4 else (1.0, 1.0, 1.0)
    else:
        s2, nug, nu = th.sigma2, th.nugget, th.nu
        rg = getattr(th, "range", None) or th.beta
        an = getattr(th, "aniso", (1.0, 1.0, 1.0))
    an = tuple(an) + (1.0,) * (3 - len(an))
    return L.Theta(float(s2), float(rg), float(nug), float(nu), (ctypes.c_double * 3)(*an))


ENGINES = {"mfma": L.ENGINE_MFMA, "tiles": L.ENGINE_TILES, "mfma_wg": L.ENGINE_MFMA_WG}


def tile_config(cfg: int, engine: str = "mfma"):
    """(R, G) of a size-class configuration."""
    r, g = ctypes.c_int32(0), ctypes.c_int32(0)
    L.check(L.lib().vecchia_tile_config(ENGINES[engine], cfg, ctypes.byref(r), ctypes.byref(g)),
            "vecchia_tile_config")
    return r.value, g.value


def permute_rows(src: torch.Tensor, perm: torch.Tensor) -> torch.Tensor:
    """dst[i] = src[perm[i]] (rows), done by the library's gather kernel."""
    _dev_check(src, perm)
    d = 1 if src.dim() == 1 else src.shape[1]
    dst = torch.empty_like(src)
    L.check(L.lib().vecchia_permute(_p(src), src.shape[0], d, _p(perm), _p(dst), _stream(src.device)),
            "vecchia_permute")
    return dst


def blocks(locs: torch.Tensor, bc: int, init_idx: torch.Tensor, block_perm: torch.Tensor,
           metric_scale: Optional[Sequence[float]] = None, max_iter: int = 30):
    """K-means blocks in random order.  Returns (perm int64[n], block_ptr int32[bc'+1], iters)."""
    _dev_check(locs, init_idx, block_perm)
    n, d = locs.shape
    lib = L.lib()
    ws = torch.empty(int(lib.vecchia_blocks_workspace_size(n, bc, d)), dtype=torch.uint8, device=locs.device)
    perm = torch.empty(n, dtype=torch.int64, device=locs.device)
    bp = torch.empty(bc + 1, dtype=torch.int32, device=locs.device)
    bc_out = ctypes.c_int64(0)
    iters = ctypes.c_int32(0)
    ms = (ctypes.c_double * d)(*metric_scale) if metric_scale is not None else None
    L.check(lib.vecchia_blocks(_p(locs), n, d, ms, _p(init_idx), _p(block_perm), bc, max_iter, _p(perm), _p(bp),
                               ctypes.byref(bc_out), ctypes.byref(iters), _p(ws), ws.numel(),
                               _stream(locs.device)), "vecchia_blocks")
    return perm, bp[: bc_out.value + 1].clone(), iters.value


def neighbors(locs_perm: torch.Tensor, block_ptr: torch.Tensor, m: int,
              metric_scale: Optional[Sequence[float]] = None):
    """Nearest earlier points of each block centroid.  Returns (nbr_ptr int32, nbr_idx int32)."""
    _dev_check(locs_perm, block_ptr)
    n, d = locs_perm.shape
    bc = block_ptr.numel() - 1
    lib = L.lib()
    cap = n * (n + 1) // 2 if m < 0 else bc * m
    cap = max(1, min(cap, 2**31 - 1))
    ws = torch.empty(int(lib.vecchia_neighbors_workspace_size(n, bc, d, m)), dtype=torch.uint8,
                     device=locs_perm.device)
    nptr = torch.empty(bc + 1, dtype=torch.int32, device=locs_perm.device)
    nidx = torch.empty(cap, dtype=torch.int32, device=locs_perm.device)
    ms = (ctypes.c_double * d)(*metric_scale) if metric_scale is not None else None
    L.check(lib.vecchia_neighbors(_p(locs_perm), n, d, ms, _p(block_ptr), bc, m, _p(nptr), _p(nidx), cap,
                                  _p(ws), ws.numel(), _stream(locs_perm.device)), "vecchia_neighbors")
    total = int(nptr[-1].item())
    return nptr, nidx[:total].clone()


ORDERS = {"morton": L.ORDER_MORTON, "maxmin": L.ORDER_MAXMIN, "hilbert": L.ORDER_HILBERT,
          "kdtree": L.ORDER_KDTREE}


def reorder_blocks(locs_perm: torch.Tensor, block_ptr: torch.Tensor, method: str,
                   metric_scale: Optional[Sequence[float]] = None):
    """Morton or maxmin order of the blocks by their centroids.  Returns
    (block_order int64[bc], point_perm int64[n] into locs_perm, block_ptr int32[bc+1])."""
    _dev_check(locs_perm, block_ptr)
    n, d = locs_perm.shape
    bc = block_ptr.numel() - 1
    lib = L.lib()
    dev = locs_perm.device
    ws = torch.empty(max(1, int(lib.vecchia_reorder_blocks_workspace_size(n, bc, d))), dtype=torch.uint8, device=dev)
    order = torch.empty(bc, dtype=torch.int64, device=dev)
    perm = torch.empty(n, dtype=torch.int64, device=dev)
    bp = torch.empty(bc + 1, dtype=torch.int32, device=dev)
    ms = (ctypes.c_double * d)(*metric_scale) if metric_scale is not None else None
    L.check(lib.vecchia_reorder_blocks(_p(locs_perm), n, d, ms, _p(block_ptr), bc, ORDERS[method], _p(order),
                                       _p(perm), _p(bp), _p(ws), ws.numel(), _stream(dev)), "vecchia_reorder_blocks")
    return order, perm, bp


class Plan:
    """Launch schedule for one block / neighbour structure (vecchia_plan_init)."""

    def __init__(self, block_ptr: torch.Tensor, nbr_ptr: torch.Tensor, n: int, max_theta: int = 1,
                 engine: str = "mfma", predict: bool = False, aux_bytes: int | None = None):
        """aux_bytes: cap on the auxiliary workspace (default: what the plan
        asks for); a smaller one runs the adjoint in more launches."""
        _dev_check(block_ptr, nbr_ptr)
        if block_ptr.dtype != torch.int32 or nbr_ptr.dtype != torch.int32:
            raise ValueError("block_ptr / nbr_ptr must be int32")
        lib = L.lib()
        bc = block_ptr.numel() - 1
        self.ws = torch.empty(int(lib.vecchia_plan_workspace_size(bc, max_theta)), dtype=torch.uint8,
                              device=block_ptr.device)
        self.c = L.Plan()
        flags = ENGINES[engine] | (L.PLAN_PREDICT if predict else 0)
        L.check(lib.vecchia_plan_init(ctypes.byref(self.c), _p(block_ptr), _p(nbr_ptr), n, bc, max_theta,
                                      flags, _p(self.ws), self.ws.numel(), _stream(block_ptr.device)),
                "vecchia_plan_init")
        self.engine = engine
        self.aux_ws = None
        if self.c.aux_ws_bytes > 0:
            nbytes = int(self.c.aux_ws_bytes) if aux_bytes is None else min(int(aux_bytes), int(self.c.aux_ws_bytes))
            self.aux_ws = torch.empty(nbytes, dtype=torch.uint8, device=block_ptr.device)
            L.check(lib.vecchia_plan_attach_aux(ctypes.byref(self.c), _p(self.aux_ws), self.aux_ws.numel()),
                    "vecchia_plan_attach_aux")
        self.block_ptr, self.nbr_ptr = block_ptr, nbr_ptr

    def __del__(self):
        # timing records, side streams and events of the concurrent size classes
        try:
            if getattr(self, "c", None) is not None and (self.c.exec or self.c.timing):
                L.lib().vecchia_plan_destroy(ctypes.byref(self.c))
        except Exception:
            pass

    @property
    def bc(self) -> int:
        return int(self.c.bc)

    @property
    def flops_la(self) -> float:
        return float(self.c.flops_la)

    @property
    def cov_entries(self) -> float:
        return float(self.c.cov_entries)

    def set_timing(self, enable: bool) -> None:
        L.check(L.lib().vecchia_plan_set_timing(ctypes.byref(self.c), 1 if enable else 0), "vecchia_plan_set_timing")

    def timing(self, reset: bool = True):
        """Per size class: (summed ms of the main kernel launches, launch count),
        followed by the summed span of the concurrent class launches per call."""
        nb = int(self.c.nbuckets)
        ms = (ctypes.c_double * (nb + 1))()
        cnt = (ctypes.c_int64 * (nb + 1))()
        L.check(L.lib().vecchia_plan_timing(ctypes.byref(self.c), ms, cnt, 1 if reset else 0), "vecchia_plan_timing")
        return [(float(ms[q]), int(cnt[q])) for q in range(nb + 1)]

    def class_kernel(self, q: int, precision: str = "fp32", grad: bool = True) -> str:
        """Name of the kernel size class q runs (vecchia_plan_class_kernel)."""
        buf = ctypes.create_string_buffer(128)
        L.check(L.lib().vecchia_plan_class_kernel(ctypes.byref(self.c), q, PRECISIONS[precision], 1 if grad else 0,
                                                  buf, 128), "vecchia_plan_class_kernel")
        return buf.value.decode()

    def flags(self) -> torch.Tensor:
        """Per (theta, block) flags of the last evaluation (device int32 view
        [max_theta, bc] into the plan workspace): 1 FP32 guard tripped, 2 not
        positive definite, 4 re-factorised in FP64."""
        off = int(self.c.off_flag)
        nt = int(self.c.max_theta)
        return self.ws[off: off + 4 * nt * self.bc].view(torch.int32).view(nt, self.bc)

    def schedule(self) -> torch.Tensor:
        """Block ids grouped by size class (device int32 view into the plan workspace)."""
        off = int(self.c.off_sched)
        return self.ws[off: off + 4 * self.bc].view(torch.int32)

    def buckets(self):
        return [(int(self.c.bucket_cfg[q]), int(self.c.bucket_off[q + 1] - self.c.bucket_off[q]))
                for q in range(self.c.nbuckets)]


def loglik(plan: Plan, locs_perm: torch.Tensor, y_perm: torch.Tensor, nbr_idx: torch.Tensor,
           thetas: Iterable, precision: str = "fp64", want_partial: bool = False):
    """Block Vecchia log-likelihood for each theta.  Returns (loglik[ntheta] f64,
    counters[ntheta, 2] i32, partial[ntheta, bc] or None) as device tensors."""
    _dev_check(locs_perm, y_perm, nbr_idx)
    th = [make_theta(t) for t in thetas]
    nt = len(th)
    arr = (L.Theta * nt)(*th)
    dev = locs_perm.device
    out = torch.empty(nt, dtype=torch.float64, device=dev)
    cnt = torch.empty((nt, 2), dtype=torch.int32, device=dev)
    part = torch.empty((nt, plan.bc), dtype=torch.float64, device=dev) if want_partial else None
    d = 1 if locs_perm.dim() == 1 else locs_perm.shape[1]
    L.check(L.lib().vecchia_loglik(ctypes.byref(plan.c), _p(locs_perm), _p(y_perm), d, _p(plan.block_ptr),
                                   _p(plan.nbr_ptr), _p(nbr_idx), arr, nt, PRECISIONS[precision], _p(out), _p(cnt),
                                   _p(part), _stream(dev)), "vecchia_loglik")
    return out, cnt, part


def loglik_dnu(plan: Plan, locs_perm: torch.Tensor, y_perm: torch.Tensor, nbr_idx: torch.Tensor,
               thetas: Iterable, rel_step: float = 1e-4):
    """d l / d nu for each theta (FP64 central difference in the library).
    Returns dnu[ntheta] f64 as a device tensor."""
    _dev_check(locs_perm, y_perm, nbr_idx)
    th = [make_theta(t) for t in thetas]
    nt = len(th)
    arr = (L.Theta * nt)(*th)
    dev = locs_perm.device
    out = torch.empty(nt, dtype=torch.float64, device=dev)
    tmp = torch.empty(2 * nt, dtype=torch.float64, device=dev)
    d = 1 if locs_perm.dim() == 1 else locs_perm.shape[1]
    L.check(L.lib().vecchia_loglik_dnu(ctypes.byref(plan.c), _p(locs_perm), _p(y_perm), d, _p(plan.block_ptr),
                                       _p(plan.nbr_ptr), _p(nbr_idx), arr, nt, float(rel_step), _p(out), _p(tmp),
                                       _stream(dev)), "vecchia_loglik_dnu")
    return out


def loglik_grad(plan: Plan, locs_perm: torch.Tensor, y_perm: torch.Tensor, nbr_idx: torch.Tensor,
                thetas: Iterable, precision: str = "fp64", want_partial: bool = False):
    """Log-likelihood and its gradient w.r.t. (sigma2, range, nugget) for each theta.
    Returns (loglik[nt], grad[nt, 3], counters[nt, 2], partial[nt, bc] | None,
    gpartial[nt, bc, 3] | None) as device tensors."""
    _dev_check(locs_perm, y_perm, nbr_idx)
    th = [make_theta(t) for t in thetas]
    nt = len(th)
    arr = (L.Theta * nt)(*th)
    dev = locs_perm.device
    out = torch.empty(nt, dtype=torch.float64, device=dev)
    grad = torch.empty((nt, 3), dtype=torch.float64, device=dev)
    cnt = torch.empty((nt, 2), dtype=torch.int32, device=dev)
    part = torch.empty((nt, plan.bc), dtype=torch.float64, device=dev) if want_partial else None
    gpart = torch.empty((nt, plan.bc, 3), dtype=torch.float64, device=dev) if want_partial else None
    d = 1 if locs_perm.dim() == 1 else locs_perm.shape[1]
    L.check(L.lib().vecchia_loglik_grad(ctypes.byref(plan.c), _p(locs_perm), _p(y_perm), d, _p(plan.block_ptr),
                                        _p(plan.nbr_ptr), _p(nbr_idx), arr, nt, PRECISIONS[precision], _p(out),
                                        _p(grad), _p(cnt), _p(part), _p(gpart), _stream(dev)),
            "vecchia_loglik_grad")
    return out, grad, cnt, part, gpart


def loglik_grad_nu(plan: Plan, locs_perm: torch.Tensor, y_perm: torch.Tensor, nbr_idx: torch.Tensor,
                   thetas: Iterable, precision: str = "fp64", want_partial: bool = False):
    """Log-likelihood and its gradient w.r.t. (sigma2, range, nugget, nu) for
    each theta, all from the adjoint (vecchia_loglik_grad_nu).  Returns
    (loglik[nt], grad[nt, 4], counters[nt, 2], partial[nt, bc] | None,
    gpartial[nt, bc, 4] | None) as device tensors."""
    _dev_check(locs_perm, y_perm, nbr_idx)
    th = [make_theta(t) for t in thetas]
    nt = len(th)
    arr = (L.Theta * nt)(*th)
    dev = locs_perm.device
    out = torch.empty(nt, dtype=torch.float64, device=dev)
    grad = torch.empty((nt, 3), dtype=torch.float64, device=dev)
    dnu = torch.empty(nt, dtype=torch.float64, device=dev)
    cnt = torch.empty((nt, 2), dtype=torch.int32, device=dev)
    part = torch.empty((nt, plan.bc), dtype=torch.float64, device=dev) if want_partial else None
    gpart = torch.empty((nt, plan.bc, 3), dtype=torch.float64, device=dev) if want_partial else None
    gnu = torch.empty((nt, plan.bc), dtype=torch.float64, device=dev) if want_partial else None
    d = 1 if locs_perm.dim() == 1 else locs_perm.shape[1]
    L.check(L.lib().vecchia_loglik_grad_nu(ctypes.byref(plan.c), _p(locs_perm), _p(y_perm), d, _p(plan.block_ptr),
                                           _p(plan.nbr_ptr), _p(nbr_idx), arr, nt, PRECISIONS[precision], _p(out),
                                           _p(grad), _p(dnu), _p(cnt), _p(part), _p(gpart), _p(gnu), _stream(dev)),
            "vecchia_loglik_grad_nu")
    g4 = torch.cat([grad, dnu[:, None]], 1)
    gp4 = torch.cat([gpart, gnu[:, :, None]], 2) if want_partial else None
    return out, g4, cnt, part, gp4


def simulate(locs_ord: torch.Tensor, nbr_ptr: torch.Tensor, nbr_idx: torch.Tensor, theta,
             z: torch.Tensor) -> torch.Tensor:
    """Sequential Vecchia draw in the given point order (see vecchia_simulate).
    theta: one parameter vector (z: n) or a list of up to 24 (z: ntheta x n)."""
    _dev_check(locs_ord, nbr_ptr, nbr_idx, z)
    n, d = locs_ord.shape
    lib = L.lib()
    many = isinstance(theta, list)
    ths = [make_theta(t) for t in (theta if many else [theta])]
    nt = len(ths)
    arr = (L.Theta * nt)(*ths)
    nnz = int(nbr_ptr[-1].item())
    ws = torch.empty(int(lib.vecchia_simulate_workspace_size(n, nnz, nt)), dtype=torch.uint8,
                     device=locs_ord.device)
    y = torch.empty((nt, n) if many else n, dtype=torch.float64, device=locs_ord.device)
    L.check(lib.vecchia_simulate(_p(locs_ord), n, d, _p(nbr_ptr), _p(nbr_idx), arr, nt, _p(z), _p(y),
                                 _p(ws), ws.numel(), _stream(locs_ord.device)), "vecchia_simulate")
    return y


# ----------------------------------------------------------------- warm start

def variogram(locs: torch.Tensor, y: torch.Tensor, nu_slot: torch.Tensor, nbins: int = 32, hmax: float = 0.5,
              nslots: int = 3, nchunks: int = 64, shared_design: bool = False):
    """Binned semivariogram features of nsets data sets (see vecchia_variogram).
    locs: (nsets, k, 2) or (k, 2) with shared_design; y: (nsets, k).  Returns
    (features float32 (nsets, nslots*nbins), gamma float64 (nsets, nbins))."""
    _dev_check(locs, y, nu_slot)
    nsets, k = y.shape
    lib = L.lib()
    ws = torch.empty(int(lib.vecchia_variogram_workspace_size(nsets, nbins, nchunks)), dtype=torch.uint8,
                     device=y.device)
    feat = torch.empty((nsets, nslots * nbins), dtype=torch.float32, device=y.device)
    gam = torch.empty((nsets, nbins), dtype=torch.float64, device=y.device)
    stride = 0 if shared_design else k * 2
    L.check(lib.vecchia_variogram(_p(locs), stride, _p(y), k, nsets, k, nbins, hmax, _p(nu_slot), nslots, _p(feat),
                                  _p(gam), nchunks, _p(ws), ws.numel(), _stream(y.device)), "vecchia_variogram")
    return feat, gam


def gemm(A: torch.Tensor, B: torch.Tensor, C: torch.Tensor, *, ta: bool = False, tb: bool = False, bias=None,
         mask=None, Z=None, relu: bool = False, accumulate: bool = False, bf16: bool = True) -> torch.Tensor:
    """C = op(A) op(B) (+bias) with the epilogues of vecchia_gemm."""
    _dev_check(A, B, C, bias, mask, Z)
    M = A.shape[1] if ta else A.shape[0]
    K = A.shape[0] if ta else A.shape[1]
    N = B.shape[0] if tb else B.shape[1]
    L.check(L.lib().vecchia_gemm(_p(A), _p(B), _p(C), _p(bias), _p(mask), _p(Z), M, N, K, A.shape[1], B.shape[1],
                                 C.shape[1], int(ta), int(tb), int(relu), int(accumulate), int(bf16),
                                 _stream(A.device)), "vecchia_gemm")
    return C


def mse(out: torch.Tensor, target: torch.Tensor, dout: torch.Tensor, nparts: int = 8):
    _dev_check(out, target, dout)
    part = torch.empty(nparts, dtype=torch.float64, device=out.device)
    L.check(L.lib().vecchia_mse(_p(out), _p(target), out.numel(), _p(dout), _p(part), nparts, _stream(out.device)),
            "vecchia_mse")
    return part


def colsum(X: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
    _dev_check(X, out)
    L.check(L.lib().vecchia_colsum(_p(X), X.shape[0], X.shape[1], X.shape[1], _p(out), _stream(X.device)),
            "vecchia_colsum")
    return out


def adam(param: torch.Tensor, grad: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int, lr: float = 1e-3,
         beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
    _dev_check(param, grad, m, v)
    L.check(L.lib().vecchia_adam(_p(param), _p(grad), _p(m), _p(v), param.numel(), lr, beta1, beta2, eps, step,
                                 _stream(param.device)), "vecchia_adam")


# ---------------------------------------------------------------- prediction


def pred_neighbors(locs_obs: torch.Tensor, locs_new: torch.Tensor, block_ptr: torch.Tensor, m: int,
                   metric_scale: Optional[Sequence[float]] = None):
    """The m observations nearest each prediction block's centroid (every
    observation is a candidate).  Returns (nbr_ptr int32, nbr_idx int32 into locs_obs)."""
    _dev_check(locs_obs, locs_new, block_ptr)
    n_obs, d = locs_obs.shape
    n_new = locs_new.shape[0]
    bc = block_ptr.numel() - 1
    lib = L.lib()
    cap = max(1, min(bc * (n_obs if m < 0 else min(m, n_obs)), 2**31 - 1))
    ws = torch.empty(int(lib.vecchia_pred_neighbors_workspace_size(n_obs, n_new, bc, d, m)), dtype=torch.uint8,
                     device=locs_obs.device)
    nptr = torch.empty(bc + 1, dtype=torch.int32, device=locs_obs.device)
    nidx = torch.empty(cap, dtype=torch.int32, device=locs_obs.device)
    ms = (ctypes.c_double * d)(*metric_scale) if metric_scale is not None else None
    L.check(lib.vecchia_pred_neighbors(_p(locs_obs), n_obs, _p(locs_new), n_new, d, ms, _p(block_ptr), bc, m,
                                       _p(nptr), _p(nidx), cap, _p(ws), ws.numel(), _stream(locs_obs.device)),
            "vecchia_pred_neighbors")
    total = int(nptr[-1].item())
    return nptr, nidx[:total].clone()


def predict(plan: Plan, locs_obs: torch.Tensor, y_obs: torch.Tensor, locs_new: torch.Tensor,
            nbr_idx: torch.Tensor, theta, want_cov: bool = False):
    """Block Vecchia prediction (vecchia_predict) with a plan built with
    predict=True.  Returns (mean[n_new], var[n_new], cov[bc, ldc, ldc] or None)."""
    _dev_check(locs_obs, y_obs, locs_new, nbr_idx)
    dev = locs_new.device
    n_new, d = locs_new.shape
    th = make_theta(theta)
    mean = torch.empty(n_new, dtype=torch.float64, device=dev)
    var = torch.empty(n_new, dtype=torch.float64, device=dev)
    ldc = max(1, int(plan.c.lmax))
    cov = torch.empty((plan.bc, ldc, ldc), dtype=torch.float64, device=dev) if want_cov else None
    L.check(L.lib().vecchia_predict(ctypes.byref(plan.c), _p(locs_obs), _p(y_obs), _p(locs_new), d,
                                    _p(plan.block_ptr), _p(plan.nbr_ptr), _p(nbr_idx), ctypes.byref(th), _p(mean),
                                    _p(var), _p(cov), ldc, _stream(dev)), "vecchia_predict")
    return mean, var, cov


def condsim(mean: torch.Tensor, var: torch.Tensor, z: torch.Tensor, y_true: Optional[torch.Tensor] = None):
    """Univariate conditional simulation (vecchia_condsim); z is R x n.
    Returns dict of sample_mean, sample_sd, lo, hi and, with y_true, picp and mspe."""
    _dev_check(mean, var, z, y_true)
    n = mean.numel()
    r = z.shape[0]
    if z.shape != (r, n):
        raise ValueError("z must be R x n")
    dev = mean.device
    lib = L.lib()
    out = {k: torch.empty(n, dtype=torch.float64, device=dev) for k in ("sample_mean", "sample_sd", "lo", "hi")}
    stats = torch.empty(2, dtype=torch.float64, device=dev)
    ws = torch.empty(int(lib.vecchia_condsim_workspace_size(n)), dtype=torch.uint8, device=dev)
    L.check(lib.vecchia_condsim(_p(mean), _p(var), n, _p(z), r, _p(y_true), _p(out["sample_mean"]),
                                _p(out["sample_sd"]), _p(out["lo"]), _p(out["hi"]), _p(stats), _p(ws), ws.numel(),
                                _stream(dev)), "vecchia_condsim")
    if y_true is not None:
        st = stats.cpu()
        out["picp"], out["mspe"] = float(st[0]), float(st[1])
    return out
