"""Block Vecchia model on one device: preprocessing (K-means blocks in random
order, nearest-neighbour conditioning sets), a launch plan, and likelihood /
gradient evaluation through the HIP library; a torch.autograd.Function exposes
the adjoint gradient to optimisers."""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np
import torch

from . import api


class BlockVecchia:
    """Data set prepared for repeated block Vecchia evaluations.

    locs: n x d (original order), y: n.  init_idx / block_perm are the
    K-means start points and the random block order (drawn by the caller).
    ordering: "random" (that order), "morton", "hilbert", "kdtree" or "maxmin"
    (block centroids).
    aniso: per-axis range multipliers; neighbour search and K-means use the
    metric 1/aniso.  nu is fixed per model: 0.5, 1.5, 2.5 in closed form, any
    other value in [0.05, 10] through the Bessel form (engine "mfma")."""

    def __init__(self, locs, y, bc: int, m: int, nu: float, init_idx, block_perm,
                 aniso: Sequence[float] = (1.0, 1.0, 1.0), kmeans_iters: int = 30, max_theta: int = 1,
                 device: str = "cuda", engine: str = "mfma", ordering: str = "random"):
        dev = torch.device(device)
        def t(a, dt):
            a = a if isinstance(a, torch.Tensor) else torch.as_tensor(np.asarray(a))
            return a.to(device=dev, dtype=dt).contiguous()
        locs_t = t(locs, torch.float64)
        y_t = t(y, torch.float64)
        self.n, self.d = locs_t.shape
        self.nu = float(nu)
        self.aniso = tuple(float(a) for a in aniso) + (1.0,) * (3 - len(aniso))
        self.metric = [1.0 / a for a in self.aniso[: self.d]]
        self.perm, self.block_ptr, self.kmeans_iters = api.blocks(
            locs_t, bc, t(init_idx, torch.int64), t(block_perm, torch.int64), self.metric, kmeans_iters)
        if ordering != "random":
            lp = api.permute_rows(locs_t, self.perm)
            _, pp, self.block_ptr = api.reorder_blocks(lp, self.block_ptr, ordering, self.metric)
            self.perm = self.perm[pp]   # compose: block order -> original index
        self.locs_perm = api.permute_rows(locs_t, self.perm)
        self.y_perm = api.permute_rows(y_t, self.perm)
        self.nbr_ptr, self.nbr_idx = api.neighbors(self.locs_perm, self.block_ptr, m, self.metric)
        if self.nbr_idx.numel() == 0:
            self.nbr_idx = torch.zeros(1, dtype=torch.int32, device=dev)
        self.plan = api.Plan(self.block_ptr, self.nbr_ptr, self.n, max_theta, engine)

    @classmethod
    def from_prepared(cls, locs_perm, y_perm, block_ptr, nbr_ptr, nbr_idx, nu, aniso=(1.0, 1.0, 1.0),
                      max_theta: int = 1, engine: str = "mfma"):
        """Wrap device tensors that are already in block order."""
        self = cls.__new__(cls)
        self.locs_perm, self.y_perm = locs_perm, y_perm
        self.block_ptr, self.nbr_ptr = block_ptr, nbr_ptr
        self.nbr_idx = nbr_idx if nbr_idx.numel() else torch.zeros(1, dtype=torch.int32, device=locs_perm.device)
        self.n, self.d = locs_perm.shape
        self.nu = float(nu)
        self.aniso = tuple(float(a) for a in aniso) + (1.0,) * (3 - len(aniso))
        self.metric = [1.0 / a for a in self.aniso[: self.d]]
        self.perm = None
        self.plan = api.Plan(block_ptr, nbr_ptr, self.n, max_theta, engine)
        return self

    def theta(self, sigma2: float, range_: float, nugget: float, nu: Optional[float] = None):
        return (float(sigma2), float(range_), float(nugget), self.nu if nu is None else float(nu), self.aniso)

    def predict(self, locs_new, bc: int, m: int, theta, init_idx, block_perm, want_cov: bool = False,
                kmeans_iters: int = 30):
        """Block Vecchia prediction (Alg. 2) at new locations (original order):
        K-means blocks of the new points, the m nearest observations of each
        block, conditional means and variances.  Returns (mean, var, cov or
        None, perm, block_ptr): mean and var in the block order of the new
        points, perm[i] = original index of the i-th, cov per block."""
        dev = self.locs_perm.device
        ln = torch.as_tensor(np.asarray(locs_new) if not isinstance(locs_new, torch.Tensor) else locs_new)
        ln = ln.to(device=dev, dtype=torch.float64).contiguous()
        k = ln.shape[0]
        perm, bp, _ = api.blocks(ln, bc, torch.as_tensor(np.asarray(init_idx), device=dev, dtype=torch.int64),
                                 torch.as_tensor(np.asarray(block_perm), device=dev, dtype=torch.int64),
                                 self.metric, kmeans_iters)
        lnp = api.permute_rows(ln, perm)
        npt, nid = api.pred_neighbors(self.locs_perm, lnp, bp, m, self.metric)
        if nid.numel() == 0:
            nid = torch.zeros(1, dtype=torch.int32, device=dev)
        plan = api.Plan(bp, npt, k, 1, "mfma", predict=True)
        mean, var, cov = api.predict(plan, self.locs_perm, self.y_perm, lnp, nid, theta, want_cov)
        return mean, var, cov, perm, bp

    def loglik(self, thetas, precision: str = "fp64", want_partial: bool = False):
        return api.loglik(self.plan, self.locs_perm, self.y_perm, self.nbr_idx, thetas, precision, want_partial)

    def loglik_grad(self, thetas, precision: str = "fp64", want_partial: bool = False):
        return api.loglik_grad(self.plan, self.locs_perm, self.y_perm, self.nbr_idx, thetas, precision,
                               want_partial)


    def loglik_grad_nu(self, thetas, precision: str = "fp64", want_partial: bool = False):
        return api.loglik_grad_nu(self.plan, self.locs_perm, self.y_perm, self.nbr_idx, thetas, precision,
                                  want_partial)

    def loglik_dnu(self, thetas, rel_step: float = 1e-4):
        return api.loglik_dnu(self.plan, self.locs_perm, self.y_perm, self.nbr_idx, thetas, rel_step)


class VecchiaLogLik(torch.autograd.Function):
    """l(sigma2, range, nugget) with the hand-written adjoint as its backward.
    The forward evaluates value and gradient in one pass of the library (no
    factors are kept); backward scales the stored 3-vector."""

    @staticmethod
    def forward(ctx, params: torch.Tensor, model: BlockVecchia, precision: str = "fp64"):
        p = params.detach().to(torch.float64).cpu().tolist()
        ll, g, cnt, _, _ = model.loglik_grad([model.theta(*p)], precision)
        ctx.save_for_backward(g[0].to(params.device, params.dtype))
        ctx.counters = cnt
        return ll[0].to(params.device, params.dtype)

    @staticmethod
    def backward(ctx, gout):
        (g,) = ctx.saved_tensors
        return gout * g, None, None


def vecchia_loglik(params: torch.Tensor, model: BlockVecchia, precision: str = "fp64") -> torch.Tensor:
    return VecchiaLogLik.apply(params, model, precision)


class VecchiaLogLikNu(torch.autograd.Function):
    """l(sigma2, range, nugget, nu) with all four derivatives from the
    library's adjoint (d l / d nu through d K_nu / d nu in the contraction)."""

    @staticmethod
    def forward(ctx, params: torch.Tensor, model: BlockVecchia, precision: str = "fp64"):
        p = params.detach().to(torch.float64).cpu().tolist()
        th = model.theta(*p)
        ll, g, cnt, _, _ = model.loglik_grad_nu([th], precision)
        ctx.save_for_backward(g[0].to(params.device, params.dtype))
        ctx.counters = cnt
        return ll[0].to(params.device, params.dtype)

    @staticmethod
    def backward(ctx, gout):
        (g,) = ctx.saved_tensors
        return gout * g, None, None


def vecchia_loglik_nu(params: torch.Tensor, model: BlockVecchia, precision: str = "fp64") -> torch.Tensor:
    return VecchiaLogLikNu.apply(params, model, precision)
