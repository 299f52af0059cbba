"""Block Vecchia log-likelihood and its reference quantities, numpy FP64.

* block_term is the definition of one factor of eq. (vecchia-vector): the
  conditional log-density log p(y_B | y_N), written as the joint Gaussian
  log-density of y_J, J = N u B, minus that of y_N, each by its own dense
  Cholesky factorisation.  Alg. 1 reaches the same value (up to rounding
  order) through its Cholesky / triangular-solve / Schur chain; the oracle
  does not follow that chain.
* loglik sums the per-block terms in block order.
* exact_loglik is eq. (likeli) through the library's log-determinant and
  linear solve (no Cholesky code shared with block_term).
* classic_vecchia_loglik is the univariate Vecchia product (Section 1), an
  independent point-wise loop used for the block-size-1 check.
* grad_trace is the textbook Gaussian log-density gradient applied to each
  block's joint and neighbour densities.
* grad_nu_trace is the same trace formula for the smoothness nu, with
  d C / d nu from the integral form of d K_nu / d nu (matern.drho_dnu).
* kl_divergence is eq. (kl-gaussian-vecchia).
"""
from __future__ import annotations

import numpy as np
from scipy import linalg

from . import matern
from .matern import LOG_2PI


def _logpdf(s, y, theta) -> float:
    """log N(y; 0, K(theta)) of the points s: one dense Cholesky K = L L^T,
    w = L^-1 y, log N = -|s| log(2 pi) / 2 - sum log diag L - w^T w / 2."""
    K = matern.cov(s, s, theta, same=True)
    L = np.linalg.cholesky(K)
    w = linalg.solve_triangular(L, y, lower=True)
    return -0.5 * y.size * LOG_2PI - float(np.sum(np.log(np.diag(L)))) - 0.5 * float(w @ w)


def block_term(s_b, y_b, s_nn, y_nn, theta) -> float:
    """One factor of eq. (vecchia-vector), log p(y_B | y_N) =
    log N(y_J; 0, K_J) - log N(y_N; 0, K_N) with J = N u B.  s_b: l x d block
    locations, s_nn: m x d neighbour locations (m may be 0: then the block's
    marginal density)."""
    sj = np.vstack([s_nn, s_b]) if s_nn.shape[0] else s_b
    yj = np.concatenate([y_nn, y_b]) if s_nn.shape[0] else y_b
    v = _logpdf(sj, yj, theta)
    if s_nn.shape[0]:
        v -= _logpdf(s_nn, y_nn, theta)
    return v


def block_terms(locs_perm, y_perm, block_ptr, nbr_ptr, nbr_idx, theta, blocks=None) -> np.ndarray:
    """Per-block log-likelihood terms l_i (block order)."""
    bc = block_ptr.size - 1
    sel = range(bc) if blocks is None else blocks
    out = []
    for i in sel:
        a, b = int(block_ptr[i]), int(block_ptr[i + 1])
        nn = nbr_idx[nbr_ptr[i]:nbr_ptr[i + 1]]
        out.append(block_term(locs_perm[a:b], y_perm[a:b], locs_perm[nn], y_perm[nn], theta))
    return np.array(out)


def loglik(locs_perm, y_perm, block_ptr, nbr_ptr, nbr_idx, theta) -> float:
    """Sum of the block terms in block order, eq. (vecchia-vector)."""
    t = block_terms(locs_perm, y_perm, block_ptr, nbr_ptr, nbr_idx, theta)
    acc = 0.0
    for v in t:
        acc += v
    return acc


def exact_loglik(locs, y, theta) -> float:
    """eq. (likeli): -n log(2 pi) / 2 - log det(K) / 2 - y^T K^-1 y / 2, with the
    library's log-determinant (LU) and linear solve."""
    n = locs.shape[0]
    K = matern.cov(locs, locs, theta, same=True)
    sign, logdet = np.linalg.slogdet(K)
    if sign <= 0:
        return float("nan")
    return -0.5 * n * LOG_2PI - 0.5 * logdet - 0.5 * float(y @ np.linalg.solve(K, y))


def classic_vecchia_loglik(locs_ordered, y_ordered, nbrs, theta) -> float:
    """Univariate Vecchia: sum_i log N(y_i; mu_i, s_i) with mu_i, s_i the
    conditional mean/variance given y_{N(i)} (N(i) = list of earlier indices).
    Independent of Alg. 1: uses a linear solve, not Cholesky/TRSM."""
    acc = 0.0
    for i in range(locs_ordered.shape[0]):
        nn = np.asarray(nbrs[i], dtype=np.int64)
        kii = theta.sigma2 + theta.nugget
        if nn.size:
            Knn = matern.cov(locs_ordered[nn], locs_ordered[nn], theta, same=True)
            kni = matern.cov(locs_ordered[nn], locs_ordered[i:i + 1], theta)[:, 0]
            coef = np.linalg.solve(Knn, kni)
            mu = coef @ y_ordered[nn]
            var = kii - coef @ kni
        else:
            mu, var = 0.0, kii
        r = y_ordered[i] - mu
        acc += -0.5 * (np.log(var) + r * r / var + LOG_2PI)
    return acc


def _logpdf_grad(s, y, theta):
    """Gradient of log N(y; 0, K(theta)) w.r.t. (sigma2, beta, nugget):
    0.5 tr[(alpha alpha^T - K^-1) dK], alpha = K^-1 y."""
    K = matern.cov(s, s, theta, same=True)
    Kinv = np.linalg.inv(K)
    alpha = Kinv @ y
    W = np.outer(alpha, alpha) - Kinv
    return np.array([0.5 * float(np.sum(W * dk)) for dk in matern.dcov(s, s, theta, same=True)])


def grad_trace(locs_perm, y_perm, block_ptr, nbr_ptr, nbr_idx, theta, blocks=None) -> np.ndarray:
    """Per-block gradient rows (bc x 3) of l_i = log p(y_J) - log p(y_N)."""
    bc = block_ptr.size - 1
    sel = range(bc) if blocks is None else blocks
    out = []
    for i in sel:
        a, b = int(block_ptr[i]), int(block_ptr[i + 1])
        nn = np.asarray(nbr_idx[nbr_ptr[i]:nbr_ptr[i + 1]], dtype=np.int64)
        J = np.concatenate([nn, np.arange(a, b)])
        g = _logpdf_grad(locs_perm[J], y_perm[J], theta)
        if nn.size:
            g = g - _logpdf_grad(locs_perm[nn], y_perm[nn], theta)
        out.append(g)
    return np.array(out)


def _logpdf_dnu(s, y, theta) -> float:
    """d/dnu of log N(y; 0, K(theta)): 0.5 tr[(alpha alpha^T - K^-1) dK/dnu]."""
    K = matern.cov(s, s, theta, same=True)
    Kinv = np.linalg.inv(K)
    alpha = Kinv @ y
    W = np.outer(alpha, alpha) - Kinv
    return 0.5 * float(np.sum(W * matern.dcov_dnu(s, s, theta)))


def grad_nu_trace(locs_perm, y_perm, block_ptr, nbr_ptr, nbr_idx, theta, blocks=None) -> np.ndarray:
    """Per-block d l_i / d nu of l_i = log p(y_J) - log p(y_N)."""
    bc = block_ptr.size - 1
    sel = range(bc) if blocks is None else blocks
    out = []
    for i in sel:
        a, b = int(block_ptr[i]), int(block_ptr[i + 1])
        nn = np.asarray(nbr_idx[nbr_ptr[i]:nbr_ptr[i + 1]], dtype=np.int64)
        J = np.concatenate([nn, np.arange(a, b)])
        g = _logpdf_dnu(locs_perm[J], y_perm[J], theta)
        if nn.size:
            g -= _logpdf_dnu(locs_perm[nn], y_perm[nn], theta)
        out.append(g)
    return np.array(out)


def kl_divergence(locs_perm, block_ptr, nbr_ptr, nbr_idx, theta) -> float:
    """eq. (kl-gaussian-vecchia): exact l(theta; 0) - block Vecchia l(theta; 0)."""
    y0 = np.zeros(locs_perm.shape[0])
    return exact_loglik(locs_perm, y0, theta) - loglik(locs_perm, y0, block_ptr, nbr_ptr, nbr_idx, theta)


def dense_vecchia_precision(locs_perm, block_ptr, nbr_ptr, nbr_idx, theta) -> np.ndarray:
    """Implied precision matrix of the block Vecchia density (tiny n only):
    y_B = A_B y_N + e_B, e_B ~ N(0, S_B) gives Q = (I-A)^T S^-1 (I-A)."""
    n = locs_perm.shape[0]
    A = np.zeros((n, n))
    Sinv = np.zeros((n, n))
    for i in range(block_ptr.size - 1):
        a, b = int(block_ptr[i]), int(block_ptr[i + 1])
        nn = np.asarray(nbr_idx[nbr_ptr[i]:nbr_ptr[i + 1]], dtype=np.int64)
        Kbb = matern.cov(locs_perm[a:b], locs_perm[a:b], theta, same=True)
        if nn.size:
            Knn = matern.cov(locs_perm[nn], locs_perm[nn], theta, same=True)
            Kbn = matern.cov(locs_perm[a:b], locs_perm[nn], theta)
            coef = np.linalg.solve(Knn, Kbn.T).T
            A[a:b, nn] = coef
            S = Kbb - coef @ Kbn.T
        else:
            S = Kbb
        Sinv[a:b, a:b] = np.linalg.inv(S)
    IA = np.eye(n) - A
    return IA.T @ Sinv @ IA
