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
from scipy import integrate, special


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


def dk_dnu(x: float, nu: float) -> float:
    """d K_nu(x) / d nu from the integral form K_nu(x) = int_0^inf exp(-x cosh t)
    cosh(nu t) dt (a textbook representation), differentiated under the
    integral: int_0^inf t sinh(nu t) exp(-x cosh t) dt, by adaptive quadrature.
    The integrand is formed in log space so that large nu t cannot overflow."""
    def f(t):
        if t == 0.0:
            return 0.0
        lt = math.log(t) - x * math.cosh(t)
        return 0.5 * (math.exp(lt + nu * t) - math.exp(lt - nu * t))
    # cut-off T where the integrand is below exp(-745) relative to its peak:
    # x cosh T >= nu T + 800 (fixed point of T = log(2 (nu T + 800) / x))
    T = 10.0
    for _ in range(60):
        T = math.log(2.0 * (nu * T + 800.0) / x)
    val, _ = integrate.quad(f, 0.0, T, epsabs=0.0, epsrel=1e-13, limit=400)
    return val


def drho_dnu(x, nu: float):
    """d rho / d nu of rho = c(nu) x^nu K_nu(x), c(nu) = 2^(1-nu) / Gamma(nu):
    rho (log(x / 2) - psi(nu)) + c(nu) x^nu dK_nu/dnu; zero at x = 0 (rho(0) = 1
    for every nu)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    c = 2.0 ** (1.0 - nu) / special.gamma(nu)
    for idx in zip(*np.nonzero(x > 0)):
        xv = float(x[idx])
        r = c * xv ** nu * special.kv(nu, xv)
        out[idx] = r * (math.log(xv / 2.0) - special.digamma(nu)) + c * xv ** nu * dk_dnu(xv, nu)
    return out


def dcov_dnu(s1, s2, theta) -> np.ndarray:
    """d C / d nu = sigma2 d rho / d nu (the nugget does not depend on nu).
    Distinct distances are evaluated once."""
    h = scaled_dist(s1, s2, theta.aniso) / theta.beta
    u, inv = np.unique(h, return_inverse=True)
    return theta.sigma2 * drho_dnu(u, theta.nu)[inv].reshape(h.shape)


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
