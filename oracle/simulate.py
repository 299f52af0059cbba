"""Data simulators (test infrastructure for the oracle side).

* exact_gp: y = chol(K) z with a dense Cholesky (small n).
* sequential_vecchia: points in a given random order; point i draws
  y_i | y_N(i) ~ N(b_i^T y_N(i), d_i) with N(i) its sim_m nearest earlier
  points, b_i = K_NN^-1 k_Ni and d_i = k_ii - k_Ni^T b_i.  This is the
  classic Vecchia joint density (block size 1), used as the data generator.
The innovations z are inputs (drawn by the seeded generator module).
"""
from __future__ import annotations

import numpy as np

from . import matern
from .preprocess import point_neighbors


def exact_gp(locs, theta, z):
    K = matern.cov(locs, locs, theta, same=True)
    return np.linalg.cholesky(K) @ z


def sequential_vecchia(locs, theta, z, order, sim_m, jitter: float = 0.0):
    """Returns y in the ORIGINAL point order.  order: simulation order (new->old)."""
    x = locs[order]
    w = np.asarray([1.0 / a for a in theta.aniso[: locs.shape[1]]])
    ptr, idx = point_neighbors(x * w, sim_m)
    n = x.shape[0]
    ys = np.empty(n)
    kii = theta.sigma2 + theta.nugget + jitter * theta.sigma2
    for i in range(n):
        nn = idx[ptr[i]:ptr[i + 1]]
        if nn.size:
            Knn = matern.cov(x[nn], x[nn], theta, same=True) + jitter * theta.sigma2 * np.eye(nn.size)
            kni = matern.cov(x[nn], x[i:i + 1], theta)[:, 0]
            b = np.linalg.solve(Knn, kni)
            ys[i] = b @ ys[nn] + np.sqrt(kii - b @ kni) * z[i]
        else:
            ys[i] = np.sqrt(kii) * z[i]
    y = np.empty(n)
    y[order] = ys
    return y
