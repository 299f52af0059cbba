"""Pins of the oracle's block Vecchia prediction (Alg. 2) and conditional
simulation against results fixed independently of its own code: exact
kriging through the precision matrix of the joint Gaussian (block-inverse
identity) when a block conditions on every observation, interpolation of
noise-free data, the one-neighbour closed form, the joint-density identity
log p(y_B | y_N) = log p(y_J) - log p(y_N) (library multivariate-normal
log-pdf), the far-field limit, brute-force neighbour order, and the sampling
properties of the simulated intervals."""
import numpy as np
import pytest
from scipy import stats

import workloads as W
from oracle import matern, predict as PR, preprocess as P, simulate

THETAS = [
    W.Theta(1.0, 0.1, 1e-6, 0.5),
    W.Theta(1.3, 0.07, 1e-3, 1.5),
    W.Theta(0.8, 0.05, 1e-2, 2.5),
    W.Theta(1.0, 0.05, 1e-3, 2.5, (1.0, 1.0, 0.2)),
]


def _field(n_obs, n_new, theta, seed):
    d = 3 if theta.aniso[2] != 1.0 else 2
    g = W.rng(seed)
    s = g.random((n_obs + n_new, d))
    if d == 3:
        s[:, 2] *= 0.2
    y = simulate.exact_gp(s, theta, g.standard_normal(n_obs + n_new))
    return s[:n_obs], y[:n_obs], s[n_obs:], y[n_obs:], d


def _blocks(s_new, bc, theta, seed):
    d = s_new.shape[1]
    wscale = [1.0 / a for a in theta.aniso[:d]]
    labels, _ = P.kmeans(s_new, wscale, W.kmeans_init(s_new.shape[0], bc, seed))
    perm, bp = P.order_blocks(labels, W.block_permutation(bc, seed))
    return perm, bp, wscale


def _joint_cov(s_obs, s_new, theta):
    """Covariance of (y_obs, y_new): nugget on same-index pairs only."""
    s = np.vstack([s_obs, s_new])
    return matern.cov(s, s, theta, same=True)


@pytest.mark.parametrize("theta", THETAS)
def test_all_observations_give_exact_kriging(theta):
    """m = all observations: every block's mean and covariance equal the exact
    conditional of that block, obtained from the joint precision matrix:
    Sigma_B|o = inv(Q_BB), mu_B|o = -inv(Q_BB) Q_Bo y_o."""
    s_obs, y_obs, s_new, _, d = _field(70, 30, theta, 11)
    perm, bp, wscale = _blocks(s_new, 4, theta, 12)
    s_new_p = s_new[perm]
    npt, nidx = PR.pred_neighbors(s_obs, s_new_p, bp, wscale, -1)
    mean, var, covs = PR.predict(s_obs, y_obs, s_new_p, bp, npt, nidx, theta)
    n = s_obs.shape[0]
    for i in range(bp.size - 1):
        a, b = bp[i], bp[i + 1]
        C = _joint_cov(s_obs, s_new_p[a:b], theta)
        Q = np.linalg.inv(C)
        qbb = Q[n:, n:]
        sig = np.linalg.inv(qbb)
        mu = -sig @ (Q[n:, :n] @ y_obs)
        assert np.allclose(covs[i], sig, rtol=1e-8, atol=1e-10 * theta.sigma2)
        assert np.allclose(mean[a:b], mu, rtol=1e-7, atol=1e-9)
        assert np.allclose(var[a:b], np.diag(sig), rtol=1e-8, atol=1e-10)


@pytest.mark.parametrize("theta", THETAS)
def test_block_term_is_the_conditional_density(theta):
    """log N(y_B; mu, Sigma) = log N(y_J; 0, K_J) - log N(y_N; 0, K_N) for any
    y_B: the predictive distribution is the conditional of the joint."""
    s_obs, y_obs, s_new, y_new, d = _field(90, 40, theta, 21)
    perm, bp, wscale = _blocks(s_new, 5, theta, 22)
    s_new_p, y_new_p = s_new[perm], y_new[perm]
    npt, nidx = PR.pred_neighbors(s_obs, s_new_p, bp, wscale, 12)
    mean, _, covs = PR.predict(s_obs, y_obs, s_new_p, bp, npt, nidx, theta)
    for i in range(bp.size - 1):
        a, b = bp[i], bp[i + 1]
        nn = nidx[npt[i]:npt[i + 1]]
        sj = np.vstack([s_obs[nn], s_new_p[a:b]])
        kj = matern.cov(sj, sj, theta, same=True)
        kn = kj[:nn.size, :nn.size]
        yj = np.concatenate([y_obs[nn], y_new_p[a:b]])
        ref = (stats.multivariate_normal(np.zeros(yj.size), kj).logpdf(yj)
               - stats.multivariate_normal(np.zeros(nn.size), kn).logpdf(y_obs[nn]))
        got = stats.multivariate_normal(mean[a:b], covs[i]).logpdf(y_new_p[a:b])
        assert abs(got - ref) <= 1e-9 * max(1.0, abs(ref))


def test_noise_free_data_are_interpolated():
    """Nugget 0: a new location that coincides with an observed neighbour gets
    that observation as its mean and zero variance."""
    th = W.Theta(1.0, 0.1, 0.0, 1.5)
    s_obs, y_obs, s_new, _, _ = _field(60, 6, th, 31)
    s_new = s_new.copy()
    s_new[2] = s_obs[17]
    bp = np.array([0, 6])
    npt, nidx = PR.pred_neighbors(s_obs, s_new, bp, [1.0, 1.0], 20)
    assert 17 in nidx
    mean, var, _ = PR.predict(s_obs, y_obs, s_new, bp, npt, nidx, th)
    assert abs(mean[2] - y_obs[17]) <= 1e-7
    assert abs(var[2]) <= 1e-7


@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5])
def test_one_neighbour_closed_form(nu):
    th = W.Theta(1.7, 0.2, 0.05, nu)
    s_obs = np.array([[0.3, 0.4]])
    y_obs = np.array([0.8])
    s_new = np.array([[0.35, 0.47]])
    npt, nidx = np.array([0, 1]), np.array([0])
    mean, var, _ = PR.predict(s_obs, y_obs, s_new, np.array([0, 1]), npt, nidx, th)
    h = np.hypot(0.05, 0.07) / th.beta
    r = {0.5: np.exp(-h), 1.5: (1 + h) * np.exp(-h), 2.5: (1 + h + h * h / 3) * np.exp(-h)}[nu]
    c0 = th.sigma2 + th.nugget
    assert mean[0] == pytest.approx(th.sigma2 * r / c0 * 0.8, rel=1e-13)
    assert var[0] == pytest.approx(c0 - (th.sigma2 * r) ** 2 / c0, rel=1e-13)


def test_far_field_prediction_is_the_prior():
    th = W.Theta(1.2, 0.01, 0.03, 2.5)
    s_obs, y_obs, _, _, _ = _field(40, 1, W.Theta(1.2, 0.1, 0.03, 2.5), 41)
    s_obs = s_obs * 0.1
    s_new = np.array([[0.9, 0.9], [0.95, 0.9]])
    npt, nidx = PR.pred_neighbors(s_obs, s_new, np.array([0, 2]), [1.0, 1.0], 10)
    mean, var, covs = PR.predict(s_obs, y_obs, s_new, np.array([0, 2]), npt, nidx, th)
    assert np.all(np.abs(mean) < 1e-20)
    assert np.allclose(covs[0], matern.cov(s_new, s_new, th, same=True), rtol=1e-14, atol=1e-300)


def test_prediction_neighbours_brute_force():
    """Exact (distance, index) order over all observations, the tree path
    equal to brute force, nested in m."""
    g = W.rng(51)
    s_obs = g.random((3000, 2))
    s_new = g.random((400, 2))
    bp = np.arange(0, 401, 8)
    c = P.block_centroids(s_new, bp, [1.0, 1.0])
    npt, nidx = PR.pred_neighbors(s_obs, s_new, bp, [1.0, 1.0], 30)
    for i in range(bp.size - 1):
        row = nidx[npt[i]:npt[i + 1]]
        d2 = ((c[i] - s_obs) ** 2).sum(1)
        o = np.lexsort((np.arange(3000), d2))[:30]
        assert np.array_equal(row, o)
    npt2, nidx2 = PR.pred_neighbors(s_obs, s_new, bp, [1.0, 1.0], 12)
    for i in range(bp.size - 1):
        assert np.array_equal(nidx2[npt2[i]:npt2[i + 1]], nidx[npt[i]:npt[i] + 12])
    # the KD-tree path (large problems) gives the same rows
    big = np.tile(s_obs, (20, 1)) + 1e-3 * g.random((60000, 2))
    bp2 = np.arange(0, 401, 1)
    assert (bp2.size - 1) * big.shape[0] > 20_000_000
    a1, b1 = PR.pred_neighbors(big, s_new, bp2, [1.0, 1.0], 25)
    cen = P.block_centroids(s_new, bp2, [1.0, 1.0])
    for i in range(0, 400, 37):
        d2 = ((cen[i] - big) ** 2).sum(1)
        assert np.array_equal(b1[a1[i]:a1[i + 1]], np.lexsort((np.arange(60000), d2))[:25])


def test_conditional_simulation_statistics():
    """Hand example (R = 2), then sampling properties: with truths drawn from
    the predictive distributions themselves the 95 % intervals cover about
    95 % of them and the MSPE is about the mean predictive variance."""
    out = PR.condsim_stats(np.array([1.0, -2.0]), np.array([4.0, 0.25]), np.array([[1.0, 0.0], [-1.0, 2.0]]),
                           np.array([1.0, 0.0]))
    assert np.allclose(out["sample_mean"], [1.0, -1.5])
    assert np.allclose(out["sample_sd"], [np.sqrt(8.0), np.sqrt(0.5)])
    assert out["picp"] == 0.5      # 1.0 inside [1 -/+ 5.5], 0.0 outside [-1.5 -/+ 1.39]
    assert out["mspe"] == pytest.approx((0.0 + 2.25) / 2)
    g = W.rng(61)
    n, r = 20000, 1000
    mean = g.normal(size=n)
    var = g.uniform(0.2, 2.0, size=n)
    y = mean + np.sqrt(var) * g.standard_normal(n)
    out = PR.condsim_stats(mean, var, g.standard_normal((r, n)), y)
    assert abs(out["picp"] - 0.95) < 0.006
    assert out["mspe"] == pytest.approx(var.mean(), rel=0.03)
