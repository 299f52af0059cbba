"""Pins of the oracle's block Vecchia log-likelihood and gradient against
results the mathematics fixes independently of the oracle's own code:
the exact GP density (eq. (likeli)) when every block conditions on all
earlier points (eq. (bv)), classic Vecchia at block size 1, permutation
invariance inside blocks, the conditional form of each block term (library
multivariate-normal log-pdf of y_B with the conditional mean and Schur
complement from library solves), KL properties (eq. (kl-gaussian-vecchia)),
and finite differences of the log-likelihood for the gradient."""
import numpy as np
import pytest
from scipy import stats

import workloads as W
from oracle import coracle, loglik as OL, matern, preprocess as P, simulate

THETAS = [
    W.Theta(1.0, 0.1, 1e-6, 0.5),
    W.Theta(1.3, 0.07, 1e-3, 1.5),
    W.Theta(0.8, 0.05, 1e-2, 2.5),
    W.Theta(1.0, 0.05, 1e-3, 2.5, (1.0, 1.0, 0.2)),
]


def _problem(n, bc, m, theta, seed=5, d=None):
    d = d or (3 if theta.aniso[2] != 1.0 else 2)
    g = W.rng(seed)
    s = g.random((n, d))
    if d == 3:
        s[:, 2] *= 0.2
    y = simulate.exact_gp(s, theta, g.standard_normal(n))
    wscale = [1.0 / a for a in theta.aniso[:d]]
    pre = P.preprocess(s, wscale, W.kmeans_init(n, bc, seed), W.block_permutation(bc, seed), m)
    return s, y, pre


@pytest.mark.parametrize("theta", THETAS)
def test_all_previous_conditioning_equals_exact_gp(theta):
    s, y, pre = _problem(120, 12, -1, theta)
    lp = pre["locs_perm"]
    yp = y[pre["perm"]]
    ex = OL.exact_loglik(lp, yp, theta)
    bv_np = OL.loglik(lp, yp, pre["block_ptr"], pre["nbr_ptr"], pre["nbr_idx"], theta)
    bv_c = coracle.loglik(lp, yp, pre["block_ptr"], pre["nbr_ptr"], pre["nbr_idx"], theta)
    assert bv_np == pytest.approx(ex, rel=1e-10)
    assert bv_c == pytest.approx(ex, rel=1e-10)
    # the exact value does not depend on the point order either
    assert OL.exact_loglik(s, y, theta) == pytest.approx(ex, rel=1e-11)


def test_exact_gp_matches_library_logpdf():
    theta = THETAS[1]
    s, y, _ = _problem(80, 8, 5, theta)
    K = matern.cov(s, s, theta, same=True)
    ref = stats.multivariate_normal(mean=np.zeros(len(y)), cov=K).logpdf(y)
    assert OL.exact_loglik(s, y, theta) == pytest.approx(ref, rel=1e-11)


@pytest.mark.parametrize("theta", THETAS[:3])
def test_block_size_one_is_classic_vecchia(theta):
    n, m = 90, 7
    g = W.rng(9)
    s = g.random((n, 2))
    y = simulate.exact_gp(s, theta, g.standard_normal(n))
    order = W.point_permutation(n, 9)
    so, yo = s[order], y[order]
    bp = np.arange(n + 1, dtype=np.int64)
    nptr, nidx = P.block_neighbors(so, bp, [1.0, 1.0], m)
    nbrs = [nidx[nptr[i]:nptr[i + 1]] for i in range(n)]
    cv = OL.classic_vecchia_loglik(so, yo, nbrs, theta)
    assert OL.loglik(so, yo, bp, nptr, nidx, theta) == pytest.approx(cv, rel=1e-11)
    assert coracle.loglik(so, yo, bp, nptr, nidx, theta) == pytest.approx(cv, rel=1e-11)


def test_permutation_within_blocks_invariant():
    theta = THETAS[2]
    s, y, pre = _problem(300, 20, 15, theta)
    lp, yp = pre["locs_perm"], y[pre["perm"]]
    bp, nptr, nidx = pre["block_ptr"], pre["nbr_ptr"], pre["nbr_idx"]
    base = coracle.loglik(lp, yp, bp, nptr, nidx, theta)
    g = W.rng(3)
    newpos = np.arange(len(yp))
    for i in range(len(bp) - 1):
        a, b = bp[i], bp[i + 1]
        newpos[a:b] = a + g.permutation(b - a)
    lp2 = np.empty_like(lp); lp2[newpos] = lp
    yp2 = np.empty_like(yp); yp2[newpos] = yp
    nidx2 = newpos[nidx]
    # neighbour order inside a set is also irrelevant
    for i in range(len(bp) - 1):
        nidx2[nptr[i]:nptr[i + 1]] = g.permutation(nidx2[nptr[i]:nptr[i + 1]])
    assert coracle.loglik(lp2, yp2, bp, nptr, nidx2, theta) == pytest.approx(base, rel=1e-12)
    assert OL.loglik(lp2, yp2, bp, nptr, nidx2, theta) == pytest.approx(base, rel=1e-12)


def _conditional_logpdf(lp, yp, nn, blk, theta):
    """log N(y_B; mu, S), mu = K_BN K_NN^-1 y_N, S = K_BB - K_BN K_NN^-1 K_NB
    (library solves and the library's multivariate-normal log-pdf)."""
    Kbb = matern.cov(lp[blk], lp[blk], theta, same=True)
    if len(nn) == 0:
        return stats.multivariate_normal(np.zeros(len(blk)), Kbb).logpdf(yp[blk])
    Knn = matern.cov(lp[nn], lp[nn], theta, same=True)
    Kbn = matern.cov(lp[blk], lp[nn], theta)
    C = np.linalg.solve(Knn, Kbn.T)
    mu = C.T @ yp[nn]
    S = Kbb - Kbn @ C
    return stats.multivariate_normal(mu, 0.5 * (S + S.T)).logpdf(yp[blk])


def test_block_term_is_conditional_logpdf():
    theta = THETAS[3]
    s, y, pre = _problem(400, 25, 30, theta)
    lp, yp = pre["locs_perm"], y[pre["perm"]]
    bp, nptr, nidx = pre["block_ptr"], pre["nbr_ptr"], pre["nbr_idx"]
    terms = coracle.block_terms(lp, yp, bp, nptr, nidx, theta)
    terms_np = OL.block_terms(lp, yp, bp, nptr, nidx, theta)
    for i in (0, 1, 7, 24):
        nn = nidx[nptr[i]:nptr[i + 1]]
        blk = np.arange(bp[i], bp[i + 1])
        ref = _conditional_logpdf(lp, yp, nn, blk, theta)
        assert terms[i] == pytest.approx(ref, rel=1e-9, abs=1e-9)
        assert terms_np[i] == pytest.approx(ref, rel=1e-9, abs=1e-9)


def test_c_and_numpy_oracles_agree_c1_shape():
    w = W.C1
    s = W.locations(w)
    z = W.standard_normal(w.n, w.seed_y)
    y = simulate.exact_gp(s, w.theta, z)
    pre = P.preprocess(s, w.metric_scale, W.kmeans_init(w.n, w.bc, w.seed_kmeans),
                       W.block_permutation(w.bc, w.seed_kmeans), w.m)
    lp, yp = pre["locs_perm"], y[pre["perm"]]
    for th in W.theta_grid_c1()[::3]:
        a = coracle.loglik(lp, yp, pre["block_ptr"], pre["nbr_ptr"], pre["nbr_idx"], th)
        b = OL.loglik(lp, yp, pre["block_ptr"], pre["nbr_ptr"], pre["nbr_idx"], th)
        assert a == pytest.approx(b, rel=1e-11)


def test_kl_nonnegative_monotone_and_trace_identity():
    theta = W.Theta(1.0, 0.08, 1e-3, 1.5)
    n, bc = 80, 10
    g = W.rng(4)
    s = g.random((n, 2))
    lab, _ = P.kmeans(s, [1.0, 1.0], W.kmeans_init(n, bc, 4))
    perm, bp = P.order_blocks(lab, W.block_permutation(bc, 4))
    lp = s[perm]
    kls = []
    for m in (2, 5, 10, 20, 40):
        nptr, nidx = P.block_neighbors(lp, bp, [1.0, 1.0], m)
        kls.append(OL.kl_divergence(lp, bp, nptr, nidx, theta))
        # tr(Sigma_BV^-1 Sigma) = n, the identity behind eq. (kl-gaussian-vecchia)
        Q = OL.dense_vecchia_precision(lp, bp, nptr, nidx, theta)
        K = matern.cov(lp, lp, theta, same=True)
        assert np.trace(Q @ K) == pytest.approx(n, rel=1e-8)
    assert all(k >= -1e-9 for k in kls)
    assert all(a >= b - 1e-9 for a, b in zip(kls, kls[1:]))  # nested neighbour sets


@pytest.mark.parametrize("theta", THETAS)
def test_gradient_matches_fd_and_numpy(theta):
    s, y, pre = _problem(220, 15, 20, theta)
    lp, yp = pre["locs_perm"], y[pre["perm"]]
    args = (lp, yp, pre["block_ptr"], pre["nbr_ptr"], pre["nbr_idx"])
    g = coracle.grad(*args, theta)
    g_np = OL.grad_trace(*args, theta).sum(0)
    np.testing.assert_allclose(g, g_np, rtol=1e-9, atol=1e-9)
    fd = []
    for k, name in enumerate(("sigma2", "beta", "nugget")):
        v = getattr(theta, name)
        h = 1e-5 * v  # relative step keeps the tiny nuggets positive
        lp_ = coracle.loglik(*args, theta.replace(**{name: v + h}))
        lm_ = coracle.loglik(*args, theta.replace(**{name: v - h}))
        fd.append((lp_ - lm_) / (2 * h))
    np.testing.assert_allclose(g, fd, rtol=2e-5, atol=1e-6 * np.abs(g).max())


@pytest.mark.parametrize("nu", [0.3, 0.8, 1.0, 2.0, 3.3])
def test_general_nu_numpy_oracle(nu):
    """Any nu > 0 through the Bessel form: all-previous conditioning equals
    the exact GP density, the block term equals the conditional log-pdf
    (library solves and multivariate normal), and the trace-formula gradient
    matches central differences."""
    theta = W.Theta(1.1, 0.08, 2e-3, nu)
    s, y, pre = _problem(90, 9, -1, theta)
    lp, yp = pre["locs_perm"], y[pre["perm"]]
    args = (lp, yp, pre["block_ptr"], pre["nbr_ptr"], pre["nbr_idx"])
    assert OL.loglik(*args, theta) == pytest.approx(OL.exact_loglik(lp, yp, theta), rel=1e-11)
    s, y, pre = _problem(90, 9, 12, theta)
    lp, yp = pre["locs_perm"], y[pre["perm"]]
    args = (lp, yp, pre["block_ptr"], pre["nbr_ptr"], pre["nbr_idx"])
    terms = OL.block_terms(*args, theta)
    bp, npt, nid = pre["block_ptr"], pre["nbr_ptr"], pre["nbr_idx"]
    for i in (0, 4, 8):
        nn = nid[npt[i]:npt[i + 1]]
        ref = _conditional_logpdf(lp, yp, nn, np.arange(bp[i], bp[i + 1]), theta)
        assert terms[i] == pytest.approx(ref, rel=1e-9)
    g = OL.grad_trace(*args, theta).sum(0)
    for k, name in enumerate(("sigma2", "beta", "nugget")):
        v, h = getattr(theta, name), 1e-6 * max(getattr(theta, name), 1e-3)
        fd = (OL.loglik(*args, theta.replace(**{name: v + h})) - OL.loglik(*args, theta.replace(**{name: v - h}))) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-5, abs=1e-6)


@pytest.mark.parametrize("nu", [0.5, 1.3, 3.3])
def test_nu_gradient_matches_fd(nu):
    """d l / d nu by the trace formula (d C / d nu from the integral form of
    d K_nu / d nu) against central differences of the Cholesky-based
    log-likelihood in nu, per block."""
    theta = W.Theta(1.1, 0.08, 2e-3, nu)
    s, y, pre = _problem(120, 12, 15, theta)
    lp, yp = pre["locs_perm"], y[pre["perm"]]
    args = (lp, yp, pre["block_ptr"], pre["nbr_ptr"], pre["nbr_idx"])
    g = OL.grad_nu_trace(*args, theta)
    h = 1e-5 * nu
    fd = (OL.block_terms(*args, theta.replace(nu=nu + h)) - OL.block_terms(*args, theta.replace(nu=nu - h))) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-6 * np.abs(fd).max())
    assert abs(g.sum() - fd.sum()) <= 1e-6 * np.abs(fd).sum()
