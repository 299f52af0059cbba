"""Blocks above the one-wave limit (m_i + l_i > 175) with the adjoint: the
conditioning sizes of the paper's accuracy study (hundreds of neighbours)
and all-previous conditioning, against the oracle's per-block trace-formula
gradient and, for all-previous conditioning, against the exact GP gradient."""
import numpy as np
import pytest
import torch

import workloads as W
from cases import oracle_terms, problem
from oracle import coracle, loglik as OL

pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="the large-block adjoint is switched off: its first GPU run ended with a "
                                      "device fault whose cause has not been found")]
DEV = "cuda"


def _t(a, dt=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device=DEV)


def _model(pb, nu, aniso=(1.0, 1.0, 1.0), max_theta=1):
    from paper_2410_04477_amd.model import BlockVecchia
    return BlockVecchia.from_prepared(_t(pb["locs_perm"]), _t(pb["y_perm"]), _t(pb["block_ptr"], torch.int32),
                                      _t(pb["nbr_ptr"], torch.int32), _t(pb["nbr_idx"], torch.int32), nu, aniso,
                                      max_theta)


def _oracle_grad(pb, th):
    return coracle.grad_terms(pb["locs_perm"], pb["y_perm"], pb["block_ptr"], pb["nbr_ptr"], pb["nbr_idx"], th)


@pytest.mark.parametrize("n,bc,m,nu,d", [(2000, 80, 200, 1.5, 2), (3000, 60, 450, 2.5, 2), (2400, 60, 300, 0.5, 3)])
def test_large_block_gradient_matches_oracle(n, bc, m, nu, d):
    aniso = (1.0, 1.0, 0.3) if d == 3 else (1.0, 1.0, 1.0)
    th = W.Theta(1.1, 0.06, 2e-3, nu, aniso)
    pb = problem(f"large-grad-{m}", n, d, bc, m, th, 40 + m, ysim="block", zmax=0.3 if d == 3 else 1.0)
    mod = _model(pb, nu, aniso)
    assert mod.plan.c.nlarge > 0
    t = [mod.theta(th.sigma2, th.beta, th.nugget)]
    ref_g = _oracle_grad(pb, th)
    ref_l = oracle_terms(pb, th)
    ll, g, cnt, part, gp = mod.loglik_grad(t, "fp64", want_partial=True)
    rows = gp[0].cpu().numpy()
    err = np.abs(rows - ref_g).max(1) / np.maximum(np.abs(ref_g).max(1), 1e-300)
    print(f"m={m}: {int(mod.plan.c.nlarge)} large blocks; worst row rel err fp64 {err.max():.1e}", flush=True)
    np.testing.assert_allclose(rows, ref_g, rtol=1e-7, atol=1e-8 * np.abs(ref_g).max())
    np.testing.assert_allclose(part[0].cpu().numpy(), ref_l, rtol=1e-8, atol=1e-9)
    ll32, g32, c32, _, gp32 = mod.loglik_grad(t, "fp32", want_partial=True)
    assert np.linalg.norm(gp32[0].cpu().numpy() - ref_g) <= 1e-3 * np.linalg.norm(ref_g)
    assert abs(float(ll32[0]) - ref_l.sum()) <= 1e-4 * abs(ref_l.sum())
    # the value of the gradient call equals the value-only call
    lv = mod.loglik(t, "fp64")[0]
    assert abs(float(lv[0]) - float(ll[0])) <= 1e-12 * abs(float(ll[0]))


def test_all_previous_conditioning_gradient_equals_exact_gp():
    """Every block conditioned on all earlier points: the block Vecchia
    density is the exact GP density, so the adjoint gradient equals the
    exact GP gradient (oracle trace formula on the whole covariance)."""
    th = W.Theta(1.3, 0.1, 5e-3, 1.5)
    pb = problem("large-exact-grad", 400, 2, 20, -1, th, 17)
    mod = _model(pb, 1.5)
    assert mod.plan.c.nlarge > 0
    _, g, _, _, _ = mod.loglik_grad([mod.theta(th.sigma2, th.beta, th.nugget)], "fp64")
    n = pb["n"]
    one = (np.array([0, n]), np.array([0, 0]), np.zeros(0, dtype=np.int64))
    ref = coracle.grad_terms(pb["locs_perm"], pb["y_perm"], *one, th).sum(0)
    got = g[0].cpu().numpy()
    print(f"exact GP gradient {ref}, block Vecchia adjoint {got}", flush=True)
    assert np.linalg.norm(got - ref) <= 1e-8 * np.linalg.norm(ref)


def test_mle_at_conditioning_size_450():
    """L-BFGS with the adjoint over plans whose blocks condition on 450
    neighbours (the paper's largest conditioning size): the end point is
    stationary by the oracle's own gradient and at least as likely as the
    generating theta."""
    from paper_2410_04477_amd import mle
    th = W.Theta(1.5, 0.08, 0.01, 1.5)
    pb = problem("large-mle-450", 3000, 2, 60, 450, th, 451, ysim="block")
    mod = _model(pb, 1.5)
    assert mod.plan.c.nlarge > 0
    res = mle.fit(mod, W.C4_THETA0, "fp64", max_evals=100)
    th_hat = W.Theta(*res.theta, 1.5)
    terms = _oracle_grad(pb, th_hat)
    args = (pb["locs_perm"], pb["y_perm"], pb["block_ptr"], pb["nbr_ptr"], pb["nbr_idx"])
    ll_hat, ll_true = coracle.loglik(*args, th_hat), coracle.loglik(*args, th)
    print(f"m = 450 MLE {res.theta} after {res.evals} evaluations; oracle l {ll_hat:.4f} (truth {ll_true:.4f}); "
          f"gradient / sum|dl_i| {np.abs(terms.sum(0)) / np.abs(terms).sum(0)}", flush=True)
    assert ll_hat >= ll_true
    assert np.all(np.abs(terms.sum(0)) <= 1e-3 * np.abs(terms).sum(0))
