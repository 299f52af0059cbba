"""Pins of the oracle's simulators, variogram and MLP."""
import numpy as np
import pytest

import workloads as W
from oracle import learned as LR, matern, simulate


def test_sequential_vecchia_with_all_neighbours_is_exact_gp():
    """With sim_m >= n-1 the sequential simulator is an exact factorisation:
    y = T z with T T^T = K (linear in z, so probe with unit vectors)."""
    n = 25
    th = W.Theta(1.2, 0.2, 1e-3, 1.5)
    s = W.rng(1).random((n, 2))
    order = W.point_permutation(n, 1)
    T = np.column_stack([simulate.sequential_vecchia(s, th, e, order, n) for e in np.eye(n)])
    np.testing.assert_allclose(T @ T.T, matern.cov(s, s, th, same=True), rtol=1e-9, atol=1e-12)


def test_exact_gp_factor():
    n = 20
    th = W.Theta(0.7, 0.1, 1e-4, 2.5)
    s = W.rng(2).random((n, 2))
    T = np.column_stack([simulate.exact_gp(s, th, e) for e in np.eye(n)])
    np.testing.assert_allclose(T @ T.T, matern.cov(s, s, th, same=True), atol=1e-12)


def test_variogram_hand_example():
    # points on a line: distances 0.1, 0.2, 0.1 ; bins of width 0.5/32
    s = np.array([[0.0, 0.0], [0.1, 0.0], [0.2, 0.0]])
    y = np.array([1.0, 3.0, 0.0])
    g, c = LR.variogram(s, y)
    k1 = int(0.1 / 0.5 * 32)   # bin 6
    k2 = int(0.2 / 0.5 * 32)   # bin 12
    assert c[k1] == 2 and c[k2] == 1 and c.sum() == 3
    assert g[k1] == pytest.approx(((1 - 3) ** 2 + (3 - 0) ** 2) / 4)
    assert g[k2] == pytest.approx((1 - 0) ** 2 / 2)


@pytest.mark.parametrize("nu,slot", [(0.5, 0), (1.5, 1), (2.5, 2)])
def test_features_hand_example(nu, slot):
    # the three points above: gamma_6 = 13/4, gamma_12 = 1/2; subset variance
    # mean(y^2) - mean(y)^2 = 10/3 - 16/9 = 14/9; features = gamma * 9/14 in
    # the nu slot, zero elsewhere (96 = 3 slots x 32 bins)
    s = np.array([[0.0, 0.0], [0.1, 0.0], [0.2, 0.0]])
    y = np.array([1.0, 3.0, 0.0])
    x = LR.features(s, y, nu)
    assert x.shape == (96,)
    ref = np.zeros(96)
    ref[slot * 32 + 6] = 3.25 * 9.0 / 14.0
    ref[slot * 32 + 12] = 0.5 * 9.0 / 14.0
    np.testing.assert_allclose(x, ref, rtol=1e-14, atol=0.0)
    # shifting y leaves both the variogram and the variance unchanged;
    # scaling y by c leaves the normalised features unchanged too
    np.testing.assert_allclose(LR.features(s, 2.5 * y + 7.0, nu), ref, rtol=1e-13, atol=0.0)


def test_mlp_backward_matches_fd():
    p = LR.init_params(0, sizes=(6, 5, 4, 3))
    g = W.rng(1)
    X = g.standard_normal((7, 6))
    T = g.standard_normal((7, 3))
    out, cache = LR.forward(p, X)
    loss, grads = LR.mse_backward(p, cache, out, T)
    eps = 1e-6
    for k, P in enumerate(p):
        flat = P.reshape(-1)
        for idx in range(0, flat.size, max(1, flat.size // 5)):
            old = flat[idx]
            flat[idx] = old + eps
            lp = float(np.mean((LR.forward(p, X)[0] - T) ** 2))
            flat[idx] = old - eps
            lm = float(np.mean((LR.forward(p, X)[0] - T) ** 2))
            flat[idx] = old
            assert grads[k].reshape(-1)[idx] == pytest.approx((lp - lm) / (2 * eps), rel=1e-5, abs=1e-9)


def test_adam_first_step_is_signed_lr():
    # with bias correction, the first Adam step moves each weight by ~lr*sign(g)
    p = [np.array([1.0, -2.0])]
    gr = [np.array([0.3, -5.0])]
    out, m, v = LR.adam_step(p, gr, [np.zeros(2)], [np.zeros(2)], 1, lr=0.01)
    np.testing.assert_allclose(out[0], [1.0 - 0.01, -2.0 + 0.01], rtol=1e-6)


def test_c_block_simulator_matches_sequential_vecchia():
    """Unit blocks + nearest earlier points: the C block simulator is the
    sequential Vecchia simulator of the numpy oracle (same draws)."""
    from oracle import coracle
    from oracle.preprocess import point_neighbors
    n, m = 60, 8
    th = W.Theta(1.1, 0.15, 1e-3, 2.5)
    s = W.rng(3).random((n, 2))
    order = W.point_permutation(n, 3)
    z = W.standard_normal(n, 4)
    ref = simulate.sequential_vecchia(s, th, z, order, m)
    ptr, idx = point_neighbors(s[order], m)
    ys = coracle.simulate(s[order], np.arange(n + 1), ptr, idx, th, z)
    np.testing.assert_allclose(ys, ref[order], rtol=1e-10, atol=1e-12)


def test_bf16_round_matches_format():
    # exactly representable values are unchanged; halfway cases go to even
    assert LR.bf16_round([1.0, -2.5, 0.0])[1] == -2.5
    one_ulp = 2.0 ** -7
    assert LR.bf16_round([1.0 + one_ulp / 2])[0] == 1.0                 # tie -> even (1.0)
    assert LR.bf16_round([1.0 + 3 * one_ulp / 2])[0] == 1.0 + 2 * one_ulp  # tie -> even
    assert LR.bf16_round([1.0 + 0.6 * one_ulp])[0] == 1.0 + one_ulp
    x = W.rng(3).standard_normal(1000)
    r = LR.bf16_round(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8 * 1.0001)
