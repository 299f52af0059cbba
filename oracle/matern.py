"""Matern covariance, eq. (maternkernel), with the closed forms for
nu in {0.5, 1.5, 2.5} and the general Bessel form for any nu.

Parametrisation (pinned by Table 1): the scaled distance is x = h / beta, with
no sqrt(2 nu) factor.  The nugget tau2 is added on the diagonal of same-index
pairs only.  Anisotropy: h = ||(s_i - s_j) / aniso||, so beta is a common
range scale and the per-axis range is beta * aniso[k].
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special


def rho_general(x, nu: float):
    """2^(1-nu)/Gamma(nu) x^nu K_nu(x), with rho(0) = 1  [eq. (maternkernel)]."""
    x = np.asarray(x, dtype=np.float64)
    out = np.ones_like(x)
    pos = x > 0
    xp = x[pos]
    out[pos] = (2.0 ** (1.0 - nu) / special.gamma(nu)) * xp ** nu * special.kv(nu, xp)
    return out


def rho(x, nu: float):
    """Closed forms of the Matern correlation for half-integer nu."""
    x = np.asarray(x, dtype=np.float64)
    e = np.exp(-x)
    if nu == 0.5:
        return e
    if nu == 1.5:
        return (1.0 + x) * e
    if nu == 2.5:
        return (1.0 + x + x * x / 3.0) * e
    return rho_general(x, nu)


def drho_dbeta_general(x, beta: float, nu: float):
    """d rho(h/beta) / d beta for any nu > 0.  With the Bessel identity
    d/dx [x^nu K_nu(x)] = -x^nu K_(nu-1)(x), rho'(x) = -2^(1-nu)/Gamma(nu)
    x^nu K_(nu-1)(x), and d rho / d beta = rho'(x) * (-x / beta)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    pos = x > 0
    xp = x[pos]
    out[pos] = (xp / beta) * (2.0 ** (1.0 - nu) / special.gamma(nu)) * xp ** nu * special.kv(nu - 1.0, xp)
    return out


def drho_dbeta(x, beta: float, nu: float):
    """d rho(h/beta) / d beta = rho'(x) * (-x / beta)."""
    x = np.asarray(x, dtype=np.float64)
    e = np.exp(-x)
    if nu == 0.5:
        g = e
    elif nu == 1.5:
        g = x * e
    elif nu == 2.5:
        g = (x / 3.0) * (1.0 + x) * e
    else:
        return drho_dbeta_general(x, beta, nu)
    return (x / beta) * g


def scaled_dist(s1: np.ndarray, s2: np.ndarray, aniso) -> np.ndarray:
    """Pairwise distances ||(s1_i - s2_j) / aniso|| (un-divided by beta)."""
    s1 = np.atleast_2d(s1)
    s2 = np.atleast_2d(s2)
    a = np.asarray(aniso[: s1.shape[1]], dtype=np.float64)
    diff = (s1[:, None, :] - s2[None, :, :]) / a
    return np.sqrt(np.sum(diff * diff, axis=-1))


def cov(s1, s2, theta, same: bool = False) -> np.ndarray:
    """C(s1_i, s2_j) = sigma2 rho(h/beta) + nugget * [i == j and same set]."""
    h = scaled_dist(s1, s2, theta.aniso)
    c = theta.sigma2 * rho(h / theta.beta, theta.nu)
    if same:
        c = c + theta.nugget * np.eye(c.shape[0])
    return c


def dcov(s1, s2, theta, same: bool = False):
    """Derivatives of cov w.r.t. (sigma2, beta, nugget)."""
    h = scaled_dist(s1, s2, theta.aniso)
    x = h / theta.beta
    d_s2 = rho(x, theta.nu)
    d_be = theta.sigma2 * drho_dbeta(x, theta.beta, theta.nu)
    d_tau = np.eye(h.shape[0]) if same else np.zeros_like(h)
    return d_s2, d_be, d_tau


def effective_range_corr(beta: float, nu: float, eff_range: float) -> float:
    """Correlation at the effective range under this parametrisation (Table 1 pin)."""
    return float(rho(np.array([eff_range / beta]), nu)[0])


LOG_2PI = math.log(2.0 * math.pi)
