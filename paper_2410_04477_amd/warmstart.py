"""Learned warm start for the block Vecchia MLE.

Features: the 32-bin empirical semivariogram of a data set (subset of 4,096
points, bins on (0, 0.5]) normalised by the subset variance and placed in the
slot of the data set's smoothness nu (96 inputs).  Network: 96 -> 256 -> 256 -> 3
with ReLU; outputs are standardised (log sigma2, log range, log(nugget + 1e-4)).
Training runs on the GPU with the library's kernels only: BF16 matrix-core
GEMMs with fused bias / ReLU epilogues (FP32 accumulation and FP32 master
weights), MSE, bias column sums and Adam.  Training data sets are drawn by the
library's sequential Vecchia simulator.  The predicted theta seeds the L-BFGS
MLE; the cold start and any invalid prediction fall back to a fixed theta_0.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import api

NBINS = 32
HMAX = 0.5
NU_SLOTS = (0.5, 1.5, 2.5)
NUG_EPS = 1e-4
SIM_JITTER = 1e-8   # added to the nugget (times sigma2) when simulating: keeps
                    # smooth, long-range fields numerically positive definite in FP64
SIZES = (96, 256, 256, 3)


def targets(thetas) -> np.ndarray:
    return np.array([[math.log(t.sigma2), math.log(t.beta), math.log(t.nugget + NUG_EPS)] for t in thetas])


class MLP:
    """96 -> 256 -> 256 -> 3 ReLU network; weights (out, in) FP32 on the device."""

    def __init__(self, seed: int, device="cuda", bf16: bool = True):
        g = np.random.Generator(np.random.PCG64(seed))
        self.params: List[torch.Tensor] = []
        for a, b in zip(SIZES[:-1], SIZES[1:]):
            lim = math.sqrt(6.0 / a)
            self.params.append(torch.tensor(g.uniform(-lim, lim, (b, a)), dtype=torch.float32, device=device))
            self.params.append(torch.zeros(b, dtype=torch.float32, device=device))
        self.m = [torch.zeros_like(p) for p in self.params]
        self.v = [torch.zeros_like(p) for p in self.params]
        self.step_count = 0
        self.bf16 = bf16
        self.tmean = np.zeros(3)
        self.tstd = np.ones(3)

    def set_params(self, params: Sequence[np.ndarray]) -> None:
        for dst, src in zip(self.params, params):
            dst.copy_(torch.as_tensor(np.asarray(src), dtype=torch.float32))

    def forward(self, X: torch.Tensor):
        W1, b1, W2, b2, W3, b3 = self.params
        B = X.shape[0]
        dev = X.device
        z1 = torch.empty((B, SIZES[1]), dtype=torch.float32, device=dev)
        a1 = torch.empty_like(z1)
        z2 = torch.empty((B, SIZES[2]), dtype=torch.float32, device=dev)
        a2 = torch.empty_like(z2)
        out = torch.empty((B, SIZES[3]), dtype=torch.float32, device=dev)
        api.gemm(X, W1, a1, tb=True, bias=b1, Z=z1, relu=True, bf16=self.bf16)
        api.gemm(a1, W2, a2, tb=True, bias=b2, Z=z2, relu=True, bf16=self.bf16)
        api.gemm(a2, W3, out, tb=True, bias=b3, bf16=self.bf16)
        return out, (X, z1, a1, z2, a2)

    def backward(self, cache, dout: torch.Tensor):
        W1, b1, W2, b2, W3, b3 = self.params
        X, z1, a1, z2, a2 = cache
        g = [torch.empty_like(p) for p in self.params]
        api.gemm(dout, a2, g[4], ta=True, bf16=self.bf16)          # dW3 = dout^T a2
        api.colsum(dout, g[5])
        dz2 = torch.empty_like(z2)
        api.gemm(dout, W3, dz2, mask=z2, bf16=self.bf16)           # (dout W3) * [z2 > 0]
        api.gemm(dz2, a1, g[2], ta=True, bf16=self.bf16)
        api.colsum(dz2, g[3])
        dz1 = torch.empty_like(z1)
        api.gemm(dz2, W2, dz1, mask=z1, bf16=self.bf16)
        api.gemm(dz1, X, g[0], ta=True, bf16=self.bf16)
        api.colsum(dz1, g[1])
        return g

    def train_step(self, X: torch.Tensor, T: torch.Tensor, lr: float) -> torch.Tensor:
        out, cache = self.forward(X)
        dout = torch.empty_like(out)
        part = api.mse(out, T, dout)
        grads = self.backward(cache, dout)
        self.step_count += 1
        for p, gr, m, v in zip(self.params, grads, self.m, self.v):
            api.adam(p, gr, m, v, self.step_count, lr)
        return part

    def fit(self, feats: torch.Tensor, thetas, epochs: int = 200, batch: int = 256, lr: float = 1e-3,
            seed: int = 0, log_every: int = 0):
        """Adam on the standardised targets; returns the per-epoch mean training loss."""
        T = targets(thetas)
        self.tmean, self.tstd = T.mean(0), T.std(0) + 1e-12
        Tn = torch.tensor((T - self.tmean) / self.tstd, dtype=torch.float32, device=feats.device)
        n = feats.shape[0]
        g = np.random.Generator(np.random.PCG64(seed))
        hist = []
        for ep in range(epochs):
            order = torch.tensor(g.permutation(n), device=feats.device)
            parts = []
            for a in range(0, n - batch + 1, batch):
                idx = order[a:a + batch]
                parts.append(self.train_step(feats.index_select(0, idx).contiguous(),
                                             Tn.index_select(0, idx).contiguous(), lr))
            hist.append(float(torch.stack(parts).sum(1).mean()))
            if log_every and (ep % log_every == 0 or ep == epochs - 1):
                print(f"[warmstart] epoch {ep} loss {hist[-1]:.4f}", flush=True)
        return hist

    def predict(self, feats: torch.Tensor) -> np.ndarray:
        """theta_hat rows (sigma2, range, nugget)."""
        out, _ = self.forward(feats.contiguous())
        t = out.double().cpu().numpy() * self.tstd + self.tmean
        return np.stack([np.exp(t[:, 0]), np.exp(t[:, 1]), np.maximum(np.exp(t[:, 2]) - NUG_EPS, 0.0)], 1)


def valid_theta(th) -> bool:
    s2, rg, nug = th
    return all(math.isfinite(v) for v in th) and 1e-4 < s2 < 1e4 and 1e-4 < rg < 10.0 and 0.0 <= nug < 1e3


# ------------------------------------------------------------- data sets ---

@dataclasses.dataclass
class Design:
    """Shared locations (simulation order) and their sequential-Vecchia neighbours."""
    locs_ord: torch.Tensor
    nbr_ptr: torch.Tensor
    nbr_idx: torch.Tensor
    sub_idx: torch.Tensor      # subset used by the variogram (positions in simulation order)


def make_design(locs: np.ndarray, order: np.ndarray, sub_idx: np.ndarray, sim_m: int = 150,
                device="cuda") -> Design:
    lo = torch.tensor(locs[order], dtype=torch.float64, device=device)
    unit = torch.arange(locs.shape[0] + 1, dtype=torch.int32, device=device)
    nptr, nidx = api.neighbors(lo, unit, sim_m, [1.0, 1.0])
    inv = np.argsort(order)
    sub_pos = torch.tensor(inv[sub_idx], dtype=torch.int64, device=device)
    return Design(lo, nptr, nidx, sub_pos)


def simulate_sets(design: Design, thetas, z: torch.Tensor) -> torch.Tensor:
    """Draw len(thetas) data sets on one design (simulation order), 24 per call."""
    out = []
    for a in range(0, len(thetas), 24):
        chunk = thetas[a:a + 24]
        th = [(t.sigma2, t.beta, t.nugget + SIM_JITTER * t.sigma2, t.nu) for t in chunk]
        out.append(api.simulate(design.locs_ord, design.nbr_ptr, design.nbr_idx, th, z[a:a + len(chunk)].contiguous()))
    return torch.cat(out, 0)


def features_for(design: Design, y_sets: torch.Tensor, nus) -> torch.Tensor:
    """Variogram features of data sets on one design (shared subset)."""
    sub = design.sub_idx
    locs_sub = design.locs_ord.index_select(0, sub).contiguous()
    y_sub = y_sets.index_select(1, sub).contiguous()
    slots = torch.tensor([NU_SLOTS.index(nu) for nu in nus], dtype=torch.int32, device=y_sets.device)
    feat, _ = api.variogram(locs_sub, y_sub, slots, NBINS, HMAX, 3, shared_design=True)
    return feat


# ------------------------------------------------------------- experiment --

def run_experiment(n_train_sets: int = 4096, n_train: int = 20_000, n_designs: int = 16, n_test_sets: int = 256,
                   n_test: int = 200_000, bc_test: int = 20_000, m_test: int = 100, epochs: int = 300,
                   batch: int = 256, lr: float = 1e-3, subset: int = 4096, sim_m: int = 150,
                   precision: str = "fp32", max_evals: int = 200, seed: int = 20240, device: str = "cuda",
                   log=print) -> dict:
    """Train the warm-start network on simulated data sets and compare warm-
    and cold-started block Vecchia MLEs on held-out data sets.  Returns a
    JSON-ready summary (times, evaluations, final log-likelihoods)."""
    import workloads as W
    from . import mle
    from .model import BlockVecchia

    t0 = time.perf_counter()
    per = n_train_sets // n_designs
    feats, thetas = [], []
    for dsg in range(n_designs):
        locs = W.uniform_square(n_train, seed + dsg)
        order = W.point_permutation(n_train, seed + dsg)
        design = make_design(locs, order, W.subset_indices(n_train, subset, seed + dsg), sim_m, device)
        th = W.warm_thetas(per, seed * 7 + dsg)
        z = torch.tensor(W.rng(seed + 1000 + dsg).standard_normal((per, n_train)), device=device)
        ys = simulate_sets(design, th, z)
        ok = torch.isfinite(ys).all(1).cpu().numpy()
        feats.append(features_for(design, ys, [t.nu for t in th])[torch.tensor(ok, device=device)])
        thetas += [t for t, g in zip(th, ok) if g]
        log(f"[warmstart] design {dsg}: {int(ok.sum())}/{per} data sets")
    feats = torch.cat(feats, 0)
    t_data = time.perf_counter() - t0
    net = MLP(seed, device)
    t1 = time.perf_counter()
    hist = net.fit(feats, thetas, epochs=epochs, batch=batch, lr=lr, seed=seed, log_every=max(1, epochs // 10))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1

    rows = []
    theta0 = W.C4_THETA0
    tests = W.warm_thetas(n_test_sets, seed + 99)
    for i, th in enumerate(tests):
        locs = W.uniform_square(n_test, seed + 50_000 + i)
        order = W.point_permutation(n_test, seed + 50_000 + i)
        design = make_design(locs, order, W.subset_indices(n_test, subset, seed + 50_000 + i), sim_m, device)
        z = torch.tensor(W.standard_normal(n_test, seed + 60_000 + i), device=device)[None]
        y_ord = simulate_sets(design, [th], z)[0]
        if not bool(torch.isfinite(y_ord).all()):
            continue
        t2 = time.perf_counter()
        th_hat = tuple(float(v) for v in net.predict(features_for(design, y_ord[None], [th.nu]))[0])
        t_pred = time.perf_counter() - t2
        used_net = valid_theta(th_hat)
        start = th_hat if used_net else theta0
        y = api.permute_rows(y_ord, torch.tensor(np.argsort(order), device=device))
        mod = BlockVecchia(locs, y, bc_test, m_test, th.nu, W.kmeans_init(n_test, bc_test, seed + i),
                           W.block_permutation(bc_test, seed + i))
        rw = mle.fit(mod, start, precision, max_evals=max_evals)
        rc = mle.fit(mod, theta0, precision, max_evals=max_evals)
        llw = float(mod.loglik([mod.theta(*rw.theta)], "fp64")[0][0])
        llc = float(mod.loglik([mod.theta(*rc.theta)], "fp64")[0][0])
        rows.append(dict(nu=th.nu, truth=(th.sigma2, th.beta, th.nugget), start=start, used_net=used_net,
                         warm_theta=rw.theta, cold_theta=rc.theta, warm_evals=rw.evals, cold_evals=rc.evals,
                         warm_s=rw.seconds + t_pred, cold_s=rc.seconds, warm_loglik=llw, cold_loglik=llc,
                         warm_grad_eta=rw.grad_eta, cold_grad_eta=rc.grad_eta, warm_restarts=rw.restarts,
                         cold_restarts=rc.restarts))
        if i % 16 == 0:
            log(f"[warmstart] test {i}: warm {rw.evals} evals {rw.seconds:.2f}s ll {llw:.3f} | "
                f"cold {rc.evals} evals {rc.seconds:.2f}s ll {llc:.3f}")
    we = np.array([r["warm_evals"] for r in rows])
    ce = np.array([r["cold_evals"] for r in rows])
    ws_ = np.array([r["warm_s"] for r in rows])
    cs_ = np.array([r["cold_s"] for r in rows])
    gap = np.array([(r["warm_loglik"] - r["cold_loglik"]) / abs(r["cold_loglik"]) for r in rows])
    return {
        "train_sets": int(feats.shape[0]), "n_train": n_train, "designs": n_designs, "epochs": epochs,
        "loss_first": hist[0], "loss_last": hist[-1], "data_s": t_data, "train_s": t_train,
        "test_sets": len(rows), "n_test": n_test, "bc_test": bc_test, "m_test": m_test, "precision": precision,
        "median_evals_warm": float(np.median(we)), "median_evals_cold": float(np.median(ce)),
        "median_seconds_warm": float(np.median(ws_)), "median_seconds_cold": float(np.median(cs_)),
        "total_seconds_warm": float(ws_.sum()), "total_seconds_cold": float(cs_.sum()),
        "net_used_fraction": float(np.mean([r["used_net"] for r in rows])),
        "rel_loglik_gap_warm_minus_cold": {"min": float(gap.min()), "median": float(np.median(gap)),
                                           "max": float(gap.max())},
        "max_grad_eta_per_n": {"warm": float(max(r["warm_grad_eta"] for r in rows)),
                               "cold": float(max(r["cold_grad_eta"] for r in rows))},
        "restarted_fits": {"warm": int(sum(r["warm_restarts"] > 0 for r in rows)),
                           "cold": int(sum(r["cold_restarts"] > 0 for r in rows))},
        "rows": rows,
    }


if __name__ == "__main__":
    import argparse
    import json
    import os
    import sys

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    ap = argparse.ArgumentParser(description="train the warm-start network and compare warm vs cold MLE")
    ap.add_argument("--train-sets", type=int, default=4096)
    ap.add_argument("--n-train", type=int, default=20_000)
    ap.add_argument("--designs", type=int, default=16)
    ap.add_argument("--test-sets", type=int, default=256)
    ap.add_argument("--n-test", type=int, default=200_000)
    ap.add_argument("--bc-test", type=int, default=20_000)
    ap.add_argument("--m-test", type=int, default=100)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--out", default="")
    a = ap.parse_args()
    res = run_experiment(a.train_sets, a.n_train, a.designs, a.test_sets, a.n_test, a.bc_test, a.m_test, a.epochs,
                         precision=a.precision, log=lambda s: print(s, file=sys.stderr, flush=True))
    txt = json.dumps({k: v for k, v in res.items() if k != "rows"})
    print(txt, flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(res, fh)
