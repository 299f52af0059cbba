"""Oracle-side problem builders shared by the tests.  Every input here comes
from the seeded generators (workloads) and the oracle; nothing comes from
the HIP path."""
from __future__ import annotations

import functools

import numpy as np

import workloads as W
from oracle import coracle, preprocess as P, simulate as S


@functools.lru_cache(maxsize=None)
def problem(name: str, n: int, d: int, bc: int, m: int, theta: W.Theta, seed: int, ysim: str = "exact",
            kmeans_iters: int = 30, zmax: float = 1.0):
    """Locations, oracle blocks / neighbours, and y (block order).
    ysim: 'exact' (dense Cholesky; small n) or 'block' (block Vecchia draw on
    the oracle's own blocks and neighbours)."""
    g = W.rng(seed)
    s = g.random((n, d))
    if d == 3:
        s[:, 2] *= zmax
    wscale = [1.0 / a for a in theta.aniso[:d]]
    labels, _ = P.kmeans(s, wscale, W.kmeans_init(n, bc, seed), kmeans_iters)
    perm, bp = P.order_blocks(labels, W.block_permutation(bc, seed))
    lp = s[perm]
    nptr, nidx = P.block_neighbors(lp, bp, wscale, m)
    z = W.standard_normal(n, seed + 7)
    if ysim == "exact":
        yp = S.exact_gp(lp, theta, z)
    else:
        yp = coracle.simulate(lp, bp, nptr, nidx, theta, z)
    return dict(name=name, locs_perm=lp, y_perm=yp, block_ptr=bp, nbr_ptr=nptr, nbr_idx=nidx, perm=perm,
                wscale=wscale, theta=theta, n=n, d=d)


@functools.lru_cache(maxsize=4)
def workload_problem(w: W.Workload, ysim: str = "block", kmeans_iters: int = 30):
    """A configured workload with the oracle's own preprocessing."""
    s = W.locations(w)
    labels, _ = P.kmeans(s, w.metric_scale, W.kmeans_init(w.n, w.bc, w.seed_kmeans), kmeans_iters)
    perm, bp = P.order_blocks(labels, W.block_permutation(w.bc, w.seed_kmeans))
    lp = s[perm]
    nptr, nidx = P.block_neighbors(lp, bp, w.metric_scale, w.m)
    z = W.standard_normal(w.n, w.seed_y)
    if ysim == "exact":
        yp = S.exact_gp(lp, w.theta, z)
    else:
        yp = coracle.simulate(lp, bp, nptr, nidx, w.theta, z)
    return dict(name=w.name, locs_perm=lp, y_perm=yp, block_ptr=bp, nbr_ptr=nptr, nbr_idx=nidx, perm=perm,
                wscale=list(w.metric_scale), theta=w.theta, n=w.n, d=w.d)


def oracle_terms(pb, theta):
    return coracle.block_terms(pb["locs_perm"], pb["y_perm"], pb["block_ptr"], pb["nbr_ptr"], pb["nbr_idx"], theta)


def oracle_sum(terms) -> float:
    acc = 0.0
    for v in terms:
        acc += float(v)
    return acc


def fourier_field(locs: np.ndarray, sigma2: float, scale, nugget: float, seed: int, nfeat: int = 256) -> np.ndarray:
    """A smooth seeded random field for full-size parity inputs where the
    block Vecchia simulator would need every block's neighbours from the
    oracle: sum of nfeat random cosines with frequencies N(0, 1 / scale^2) per
    axis (variance sigma2, correlation length ~ scale), plus white noise of
    variance nugget.  Not a draw from the Matern model; any y is a valid
    likelihood input, and this one has the value range and spatial structure
    of the simulated fields."""
    g = W.rng(seed)
    d = locs.shape[1]
    om = g.standard_normal((nfeat, d)) / np.asarray(scale, dtype=np.float64)[:d]
    ph = g.uniform(0.0, 2.0 * np.pi, nfeat)
    y = np.zeros(locs.shape[0])
    for f in range(nfeat):
        y += np.cos(locs @ om[f] + ph[f])
    y *= np.sqrt(2.0 * sigma2 / nfeat)
    return y + np.sqrt(nugget) * g.standard_normal(locs.shape[0])
