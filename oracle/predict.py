"""Block Vecchia prediction (Section 2.4, Alg. 2) and the univariate
conditional simulation behind the prediction-interval coverage (PICP) and the
mean square prediction error (MSPE) of Section 3, numpy FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* pred_neighbors: for each block of new locations, the m observed points
  nearest its centroid (Alg. 2, nearest neighbours).
* predict: per block, Sigma^con, Sigma^cross, Sigma^lk (Alg. 2, covariance
  generation), then the conditional mean and covariance of the block given its
  neighbours' data (Alg. 2; the formulas of Section 2.4).
* condsim_stats: R rounds of univariate conditional simulation from the
  predicted means and the diagonals of the block covariances, the sample mean
  and standard deviation per location, the 95 % interval, PICP and MSPE.

Readings where the paper is silent or garbled:
  * Every observed point is a neighbour candidate of every prediction block
    (the observations precede the new locations), with the centroid, squared
    distance and (distance, index) tie rule of the likelihood's neighbour
    search; m_i = min(m, n); m = -1 means all observed points.
  * Alg. 2 generates Sigma^cross as cov(S_NN, S_B*) (m x l) but multiplies it
    on the left of (Sigma^con)^-1 y_NN, which needs l x m: the cross-covariance
    in the two formulas is K(B*, NN), the transpose.
  * Sigma^lk carries the nugget on its diagonal: what is predicted is a new
    noisy observation, the quantity that PICP and MSPE compare with.  Observed
    and new locations are different indices, so Sigma^cross carries none.
  * Conditional simulation: draws mu_j + sqrt(Sigma_jj) z_rj (the random
    numbers z are inputs); sample mean and sample standard deviation (divisor
    R - 1) per location; interval sample mean -/+ z_0.975 sample sd; PICP is
    the fraction of held-out true values inside their interval, MSPE the mean
    squared difference between the sample mean and the true value.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree

from . import matern
from .preprocess import _knn_one, _sqdist, block_centroids

Z975 = 1.959963984540054   # standard normal quantile at 0.975


def pred_neighbors(locs_obs: np.ndarray, locs_pred_perm: np.ndarray, block_ptr: np.ndarray, metric_scale,
                   m: int):
    """m nearest observed points of each prediction block's centroid.
    Returns (nbr_ptr, nbr_idx) as int64 CSR, rows sorted by (distance, index)."""
    w = np.asarray(metric_scale, dtype=np.float64)
    x = locs_obs * w
    n = x.shape[0]
    bc = block_ptr.size - 1
    cen = block_centroids(locs_pred_perm, block_ptr, metric_scale)
    if m < 0:
        rows = [np.arange(n, dtype=np.int64) for _ in range(bc)]
    elif bc * n <= 20_000_000:
        rows = [_knn_one(cen[i], x, min(m, n)).astype(np.int64) for i in range(bc)]
    else:
        # a KD-tree proposes candidates; the exact order is re-applied and a row
        # whose candidates are not provably complete is done by brute force
        mi = min(m, n)
        kq = min(n, 2 * mi + 16)
        dist, idx = cKDTree(x).query(cen, k=kq, workers=-1)
        idx = np.atleast_2d(idx)
        dist = np.atleast_2d(dist)
        rows = []
        for i in range(bc):
            cand = idx[i]
            d2 = _sqdist(cen[i], x[cand])
            o = np.lexsort((cand, d2))
            ok = kq == n or np.sqrt(d2[o[mi - 1]]) < dist[i][-1] * (1.0 - 1e-12)
            rows.append(cand[o[:mi]].astype(np.int64) if ok else _knn_one(cen[i], x, mi).astype(np.int64))
    counts = np.array([r.size for r in rows], dtype=np.int64)
    nbr_ptr = np.zeros(bc + 1, dtype=np.int64)
    np.cumsum(counts, out=nbr_ptr[1:])
    nbr_idx = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    return nbr_ptr, nbr_idx.astype(np.int64)


def predict_block(s_b, s_nn, y_nn, theta):
    """One block of Alg. 2: (mu_B*, Sigma_B*)."""
    sig_lk = matern.cov(s_b, s_b, theta, same=True)            # Sigma^lk (l x l)
    if s_nn.shape[0] == 0:
        return np.zeros(s_b.shape[0]), sig_lk
    sig_con = matern.cov(s_nn, s_nn, theta, same=True)         # Sigma^con (m x m)
    sig_cross = matern.cov(s_b, s_nn, theta)                   # K(B*, NN) (l x m)
    mu = sig_cross @ np.linalg.solve(sig_con, y_nn)            # conditional mean
    sigma = sig_lk - sig_cross @ np.linalg.solve(sig_con, sig_cross.T)   # conditional covariance
    return mu, sigma


def predict(locs_obs, y_obs, locs_pred_perm, block_ptr, nbr_ptr, nbr_idx, theta):
    """Alg. 2 over all blocks.  Returns (mean[n*], var[n*], covs) with the
    predictions in the block order of locs_pred_perm and covs[i] the l_i x l_i
    conditional covariance of block i."""
    ns = locs_pred_perm.shape[0]
    mean = np.empty(ns)
    var = np.empty(ns)
    covs = []
    for i in range(block_ptr.size - 1):
        a, b = int(block_ptr[i]), int(block_ptr[i + 1])
        nn = nbr_idx[nbr_ptr[i]:nbr_ptr[i + 1]]
        mu, sig = predict_block(locs_pred_perm[a:b], locs_obs[nn], y_obs[nn], theta)
        mean[a:b] = mu
        var[a:b] = np.diag(sig)
        covs.append(sig)
    return mean, var, covs


def condsim_stats(mean, var, z, y_true=None):
    """Univariate conditional simulation: z is R x n* standard normal numbers.
    Returns sample mean, sample sd, interval bounds, and (with y_true) PICP and MSPE."""
    z = np.atleast_2d(z)
    r = z.shape[0]
    draws = mean[None, :] + np.sqrt(var)[None, :] * z
    smean = draws.mean(axis=0)
    ssd = np.sqrt(((draws - smean[None, :]) ** 2).sum(axis=0) / (r - 1))
    lo = smean - Z975 * ssd
    hi = smean + Z975 * ssd
    out = dict(sample_mean=smean, sample_sd=ssd, lo=lo, hi=hi)
    if y_true is not None:
        out["picp"] = float(np.mean((y_true >= lo) & (y_true <= hi)))
        out["mspe"] = float(np.mean((smean - y_true) ** 2))
    return out
