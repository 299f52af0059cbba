"""Pins of the oracle's Matern covariance (eq. (maternkernel), Table 1)."""
import os

import numpy as np
import pytest
from scipy import special

from oracle import matern
from workloads import Theta

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table1_beta.txt")


def _bessel_form(x, nu):
    # written independently of the oracle: 2^(1-nu)/Gamma(nu) x^nu K_nu(x)
    return 2.0 ** (1 - nu) / special.gamma(nu) * x ** nu * special.kv(nu, x)


@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5])
def test_closed_forms_match_bessel(nu):
    x = np.array([1e-3, 0.05, 0.3, 1.0, 2.5, 7.0, 20.0])
    np.testing.assert_allclose(matern.rho(x, nu), _bessel_form(x, nu), rtol=1e-12)


def test_rho_at_zero_is_one():
    for nu in (0.5, 1.5, 2.5, 0.7):
        assert matern.rho(np.array([0.0]), nu)[0] == pytest.approx(1.0, abs=0)


def test_table1_pins_parametrisation():
    """All nine printed beta give the same correlation at the effective range
    only under x = h/beta (no sqrt(2 nu) factor).  The value is ~1/45."""
    rows = np.loadtxt(GOLD, comments="#")
    vals = [matern.effective_range_corr(b, nu, er) for er, nu, b in rows]
    assert np.ptp(vals) < 1e-5
    assert np.mean(vals) == pytest.approx(1.0 / 45.0, rel=2e-4)
    # the sqrt(2 nu) h / beta reading spreads the nine values apart
    alt = [float(_bessel_form(np.sqrt(2 * nu) * er / b, nu)) for er, nu, b in rows]
    assert np.ptp(alt) > 1e-2


@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5])
def test_drho_dbeta_matches_fd(nu):
    h = np.array([0.01, 0.05, 0.2, 0.6])
    beta = 0.07
    eps = 1e-7
    fd = (matern.rho(h / (beta + eps), nu) - matern.rho(h / (beta - eps), nu)) / (2 * eps)
    np.testing.assert_allclose(matern.drho_dbeta(h / beta, beta, nu), fd, rtol=1e-7)


def test_nugget_only_on_same_index_and_anisotropy():
    s = np.array([[0.1, 0.2, 0.00], [0.1, 0.2, 0.00], [0.3, 0.2, 0.01]])
    th = Theta(2.0, 0.05, 0.1, 0.5, (1.0, 1.0, 0.2))
    K = matern.cov(s, s, th, same=True)
    # duplicate location, different index: no nugget
    assert K[0, 1] == pytest.approx(2.0)
    assert K[0, 0] == pytest.approx(2.1)
    # per-axis range beta*aniso: dx = 0.2 over 0.05, dz = 0.01 over 0.01
    x = np.sqrt((0.2 / 0.05) ** 2 + (0.01 / 0.01) ** 2)
    assert K[0, 2] == pytest.approx(2.0 * np.exp(-x), rel=1e-14)


@pytest.mark.parametrize("nu", [0.2, 0.5, 0.8, 1.0, 1.5, 2.0, 2.5, 3.7])
def test_general_derivative_matches_fd_and_closed_forms(nu):
    """The Bessel form of d rho / d beta against central differences of the
    Bessel form of rho, and against the closed forms at half-integer nu."""
    h = np.array([0.003, 0.01, 0.05, 0.2, 0.6, 2.0])
    beta = 0.07
    eps = 1e-7
    fd = (matern.rho_general(h / (beta + eps), nu) - matern.rho_general(h / (beta - eps), nu)) / (2 * eps)
    got = matern.drho_dbeta_general(h / beta, beta, nu)
    np.testing.assert_allclose(got, fd, rtol=2e-6, atol=1e-12)
    if nu in (0.5, 1.5, 2.5):
        np.testing.assert_allclose(got, matern.drho_dbeta(h / beta, beta, nu), rtol=1e-12)
        np.testing.assert_allclose(matern.rho_general(h / beta, nu), matern.rho(h / beta, nu), rtol=1e-12)


def test_drho_dnu_closed_form_at_one_half():
    """At nu = 1/2, d K_nu / d nu = sqrt(pi / (2x)) E1(2x) e^x (a textbook
    special case) and psi(1/2) = -gamma - 2 log 2, so
    d rho / d nu = e^-x (log(x/2) + gamma + 2 log 2) + e^x E1(2x)."""
    x = np.array([1e-3, 0.02, 0.3, 1.0, 2.5, 7.0, 25.0])
    ref = np.exp(-x) * (np.log(x / 2) + np.euler_gamma + 2 * np.log(2.0)) + np.exp(x) * special.exp1(2 * x)
    np.testing.assert_allclose(matern.drho_dnu(x, 0.5), ref, rtol=1e-11)


@pytest.mark.parametrize("nu", [0.07, 0.3, 0.8, 1.0, 1.5, 2.2, 3.7, 7.5, 10.0])
def test_drho_dnu_matches_fd_of_library_bessel(nu):
    """The integral form of d rho / d nu against central differences in nu of
    the library's K_nu; zero at distance zero."""
    x = np.array([0.0, 1e-4, 0.01, 0.3, 1.0, 2.5, 7.0, 30.0])
    e = 1e-5 * nu
    fd = (_bessel_form(x[1:], nu + e) - _bessel_form(x[1:], nu - e)) / (2 * e)
    got = matern.drho_dnu(x, nu)
    assert got[0] == 0.0
    np.testing.assert_allclose(got[1:], fd, rtol=1e-6, atol=1e-9)
