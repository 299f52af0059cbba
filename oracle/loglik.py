"""Block Vecchia log-likelihood and its reference quantities, numpy FP64.

* block_loglik_alg1 follows Alg. 1 (correction items, then independent
  computation) step by step for one block, in the paper's notation.
* loglik sums the per-block terms in block order, as in the final loop of
  Alg. 1: l <- l - (u_i + d_i + l_i log 2 pi) / 2.
* exact_loglik is eq. (likeli) by a dense Cholesky.
* classic_vecchia_loglik is the univariate Vecchia product (Section 1), an
  independent point-wise loop used for the block-size-1 check.
* grad_trace is the textbook Gaussian log-density gradient applied to each
  block's joint and neighbour densities (the block term of eq.
  (vecchia-vector) is log p(y_J) - log p(y_N)).
* grad_nu_trace is the same trace formula for the smoothness nu, with
  d C / d nu from the integral form of d K_nu / d nu (matern.drho_dnu).
* kl_divergence is eq. (kl-gaussian-vecchia).
"""
from __future__ import annotations

import numpy as np
from scipy import linalg

from . import matern
from .matern import LOG_2PI


def _chol_lower(a: np.ndarray) -> np.ndarray:
    return np.linalg.cholesky(a)


def block_loglik_alg1(s_b, y_b, s_nn, y_nn, theta) -> float:
    """One block of Alg. 1.  s_b: l x d block locations, s_nn: m x d neighbour
    locations (m may be 0)."""
    l = s_b.shape[0]
    sig_lk = matern.cov(s_b, s_b, theta, same=True)                # Sigma^lk
    if s_nn.shape[0] > 0:
        sig_con = matern.cov(s_nn, s_nn, theta, same=True)         # Sigma^con
        sig_cross = matern.cov(s_nn, s_b, theta)                   # Sigma^cross (m x l)
        L = _chol_lower(sig_con)                                   # batchedPOTRF
        sig_cross_p = linalg.solve_triangular(L, sig_cross, lower=True)   # batchedTRSM
        y_nn_p = linalg.solve_triangular(L, y_nn, lower=True)      # batchedTRSV
        sig_cor = sig_cross_p.T @ sig_cross_p                      # batchedGEMM
        mu_cor = sig_cross_p.T @ y_nn_p                            # batchedGEMV
        sig_new = sig_lk - sig_cor                                 # elementwise
        mu_new = mu_cor
    else:
        sig_new = sig_lk
        mu_new = np.zeros(l)
    Lp = _chol_lower(sig_new)                                      # batchedPOTRF
    v = linalg.solve_triangular(Lp, y_b - mu_new, lower=True)      # batchedTRSV
    u = float(v @ v)                                               # batchedDotProduct
    d = 2.0 * float(np.sum(np.log(np.diag(Lp))))                   # 2 log det L'
    return -0.5 * (u + d + l * LOG_2PI)


def block_terms(locs_perm, y_perm, block_ptr, nbr_ptr, nbr_idx, theta, blocks=None) -> np.ndarray:
    """Per-block log-likelihood terms l_i (block order)."""
    bc = block_ptr.size - 1
    sel = range(bc) if blocks is None else blocks
    out = []
    for i in sel:
        a, b = int(block_ptr[i]), int(block_ptr[i + 1])
        nn = nbr_idx[nbr_ptr[i]:nbr_ptr[i + 1]]
        out.append(block_loglik_alg1(locs_perm[a:b], y_perm[a:b], locs_perm[nn], y_perm[nn], theta))
    return np.array(out)


def loglik(locs_perm, y_perm, block_ptr, nbr_ptr, nbr_idx, theta) -> float:
    """Sum of block terms in block order (Alg. 1, final loop)."""
    t = block_terms(locs_perm, y_perm, block_ptr, nbr_ptr, nbr_idx, theta)
    acc = 0.0
    for v in t:
        acc += v
    return acc


def exact_loglik(locs, y, theta) -> float:
    """eq. (likeli) by dense Cholesky."""
    n = locs.shape[0]
    K = matern.cov(locs, locs, theta, same=True)
    L = _chol_lower(K)
    w = linalg.solve_triangular(L, y, lower=True)
    return -0.5 * n * LOG_2PI - float(np.sum(np.log(np.diag(L)))) - 0.5 * float(w @ w)


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
