"""Matern covariance for any nu (Bessel form) on the GPU: the correlation
itself over both branches of the Bessel evaluation, then log-likelihood,
gradient and prediction against the numpy oracle (scipy's K_nu), and the
error paths."""
import numpy as np
import pytest
import torch

import workloads as W
from cases import problem
from oracle import loglik as OL, matern, predict as PR

pytestmark = pytest.mark.gpu
DEV = "cuda"
NUS = [0.3, 0.8, 1.0, 2.0, 3.7]


def _t(a, dt=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device=DEV)


@pytest.mark.parametrize("nu", [0.05, 0.3, 0.5001, 0.8, 1.0, 1.2, 2.0, 3.7, 7.5, 10.0])
def test_correlation_through_one_neighbour_prediction(nu):
    """One neighbour and one new point per block: the conditional mean is
    sigma2 rho(x) / (sigma2 + nugget) y, so it returns rho at 400 distances
    from 1e-4 to 60 range units (Temme's series below x = 2, the continued
    fraction above), compared with 2^(1-nu)/Gamma(nu) x^nu K_nu(x) from scipy."""
    from paper_2410_04477_amd import api
    th = W.Theta(1.0, 1.0, 0.0, nu)
    x = np.geomspace(1e-4, 60.0, 400)
    s_obs = np.stack([np.zeros_like(x), np.zeros_like(x)], 1)
    s_obs[:, 0] = np.arange(x.size) * 1e3   # far apart: each block sees only its own neighbour
    s_new = s_obs.copy()
    s_new[:, 1] = x
    bp = np.arange(x.size + 1)
    npt, nid = np.arange(x.size + 1), np.arange(x.size)
    plan = api.Plan(_t(bp, torch.int32), _t(npt, torch.int32), x.size, 1, "mfma", predict=True)
    mean, var, _ = api.predict(plan, _t(s_obs), _t(np.ones(x.size)), _t(s_new), _t(nid, torch.int32), th)
    rho = mean.cpu().numpy()
    ref = matern.rho_general(x, nu)
    np.testing.assert_allclose(rho, ref, rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(var.cpu().numpy(), 1.0 - ref * ref, rtol=1e-10, atol=1e-13)


def _gpu_ll(pb, thetas, precision, grad=False):
    from paper_2410_04477_amd import api
    plan = api.Plan(_t(pb["block_ptr"], torch.int32), _t(pb["nbr_ptr"], torch.int32), pb["n"], len(thetas))
    args = (plan, _t(pb["locs_perm"]), _t(pb["y_perm"]), _t(pb["nbr_idx"], torch.int32), thetas, precision)
    if grad:
        ll, g, cnt, part, gpart = api.loglik_grad(*args, want_partial=True)
        return ll.cpu().numpy(), g.cpu().numpy(), part.cpu().numpy(), gpart.cpu().numpy(), plan
    ll, cnt, part = api.loglik(*args, want_partial=True)
    return ll.cpu().numpy(), None, part.cpu().numpy(), None, plan


@pytest.mark.parametrize("m,bc", [(12, 80), (60, 80), (139, 150)])
def test_loglik_matches_numpy_oracle(m, bc):
    """FP64 per block within 1e-8 and the FP32-bulk total within 1e-4, for a
    batch mixing Bessel-form and closed-form nu (the classes span G = 4 .. 11)."""
    base = W.Theta(1.2, 0.08, 1e-3, 1.5)
    pb = problem(f"gnu{m}", 1500, 2, bc, m, base, 71 + m)
    thetas = [base.replace(nu=nu) for nu in NUS] + [base]
    ll64, _, p64, _, plan = _gpu_ll(pb, thetas, "fp64")
    ll32, _, _, _, _ = _gpu_ll(pb, thetas, "fp32")
    print("classes G", sorted(int(c) + 1 for c in plan.c.bucket_cfg[:plan.c.nbuckets]))
    args = (pb["locs_perm"], pb["y_perm"], pb["block_ptr"], pb["nbr_ptr"], pb["nbr_idx"])
    for k, th in enumerate(thetas):
        ref = OL.block_terms(*args, th)
        np.testing.assert_allclose(p64[k], ref, rtol=1e-8, atol=1e-9)
        assert abs(ll64[k] - ref.sum()) <= 1e-8 * abs(ref.sum())
        e32 = abs(ll32[k] - ref.sum()) / abs(ref.sum())
        print(f"nu={th.nu}: fp64 rel {abs(ll64[k] - ref.sum()) / abs(ref.sum()):.1e}, fp32-bulk rel {e32:.1e}")
        assert e32 <= 1e-4, (th.nu, ll32[k], ref.sum())


@pytest.mark.parametrize("nu", [0.8, 2.0])
def test_gradient_matches_numpy_oracle(nu):
    """FP64 adjoint within 1e-8 of the oracle's trace formula; FP32-bulk per
    block within 1e-3 of the scale of its terms."""
    th = W.Theta(1.2, 0.08, 1e-3, nu)
    pb = problem("gnug", 1200, 2, 60, 100, W.Theta(1.2, 0.08, 1e-3, 1.5), 77)
    args = (pb["locs_perm"], pb["y_perm"], pb["block_ptr"], pb["nbr_ptr"], pb["nbr_idx"])
    ref = OL.grad_trace(*args, th)
    _, g64, _, gp64, _ = _gpu_ll(pb, [th], "fp64", grad=True)
    _, g32, _, gp32, _ = _gpu_ll(pb, [th], "fp32", grad=True)
    assert np.linalg.norm(g64[0] - ref.sum(0)) <= 1e-8 * np.linalg.norm(ref.sum(0))
    np.testing.assert_allclose(gp64[0], ref, rtol=1e-7, atol=1e-7 * np.abs(ref).max())
    scale = np.abs(ref).sum(0)
    assert np.all(np.abs(g32[0] - ref.sum(0)) <= 1e-3 * scale)


def test_prediction_matches_oracle():
    from paper_2410_04477_amd import api
    th = W.Theta(1.1, 0.12, 2e-3, 1.3)
    g = W.rng(181)
    s_obs, s_new = g.random((800, 2)), g.random((90, 2))
    y_obs = g.standard_normal(800)
    bp = np.arange(0, 91, 9)
    npt, nid = PR.pred_neighbors(s_obs, s_new, bp, [1.0, 1.0], 40)
    mean_o, var_o, covs_o = PR.predict(s_obs, y_obs, s_new, bp, npt, nid, th)
    plan = api.Plan(_t(bp, torch.int32), _t(npt, torch.int32), 90, 1, "mfma", predict=True)
    mean, var, cov = api.predict(plan, _t(s_obs), _t(y_obs), _t(s_new), _t(nid, torch.int32), th, True)
    assert np.max(np.abs(mean.cpu().numpy() - mean_o)) <= 1e-9
    assert np.max(np.abs(var.cpu().numpy() - var_o)) <= 1e-10
    cov = cov.cpu().numpy()
    for i in range(bp.size - 1):
        assert np.max(np.abs(cov[i, :9, :9] - covs_o[i])) <= 1e-10


def test_error_paths():
    from paper_2410_04477_amd import api
    from paper_2410_04477_amd._lib import VecchiaError
    th = W.Theta(1.0, 0.1, 1e-3, 1.5)
    pb = problem("gnu-err", 400, 2, 40, 20, th, 91)
    lp, yp, nid = _t(pb["locs_perm"]), _t(pb["y_perm"]), _t(pb["nbr_idx"], torch.int32)
    bp, npt = _t(pb["block_ptr"], torch.int32), _t(pb["nbr_ptr"], torch.int32)
    plan = api.Plan(bp, npt, 400, 1)
    for nu, word in ((0.01, "unsupported"), (12.0, "unsupported"), (-1.0, "invalid"), (float("nan"), "invalid")):
        with pytest.raises(VecchiaError, match=word):
            api.loglik(plan, lp, yp, nid, [th.replace(nu=nu)])
    # the Bessel form runs on the one-wave kernels only
    tplan = api.Plan(bp, npt, 400, 1, "tiles")
    with pytest.raises(VecchiaError, match="unsupported"):
        api.loglik(tplan, lp, yp, nid, [th.replace(nu=1.0)])
    big = problem("gnu-large", 1200, 2, 40, 190, th, 93)
    lplan = api.Plan(_t(big["block_ptr"], torch.int32), _t(big["nbr_ptr"], torch.int32), 1200, 1)
    assert lplan.c.nlarge > 0
    with pytest.raises(VecchiaError, match="unsupported"):
        api.loglik(lplan, _t(big["locs_perm"]), _t(big["y_perm"]), _t(big["nbr_idx"], torch.int32),
                   [th.replace(nu=1.0)])
    # closed forms still take their own path after a Bessel-form call
    ll, _, _ = api.loglik(plan, lp, yp, nid, [th])
    ref = OL.loglik(pb["locs_perm"], pb["y_perm"], pb["block_ptr"], pb["nbr_ptr"], pb["nbr_idx"], th)
    assert abs(float(ll[0]) - ref) <= 1e-8 * abs(ref)


def test_mle_with_bessel_form():
    """L-BFGS on (sigma2, range, nugget) at nu = 1.0 (Bessel-form kernels):
    the fit is at least as likely as the truth and better than the start."""
    from paper_2410_04477_amd import mle
    from paper_2410_04477_amd.model import BlockVecchia
    th = W.Theta(1.2, 0.1, 0.01, 1.0)
    pb = problem("gnu-mle", 2000, 2, 200, 30, th, 83)
    mod = BlockVecchia.from_prepared(_t(pb["locs_perm"]), _t(pb["y_perm"]), _t(pb["block_ptr"], torch.int32),
                                     _t(pb["nbr_ptr"], torch.int32), _t(pb["nbr_idx"], torch.int32), 1.0)
    res = mle.fit(mod, (1.0, 0.05, 0.05), "fp64", max_evals=80)
    ll_true = float(mod.loglik([mod.theta(th.sigma2, th.beta, th.nugget)])[0][0])
    ll0 = float(mod.loglik([mod.theta(1.0, 0.05, 0.05)])[0][0])
    assert res.loglik >= ll_true - 1e-6 * abs(ll_true)
    assert res.loglik > ll0
    assert 0.5 < res.theta[0] / th.sigma2 < 2.0 and 0.5 < res.theta[1] / th.beta < 2.0


@pytest.mark.parametrize("nu", [0.5, 1.3, 3.7])
def test_nu_derivative_matches_oracle(nu):
    """d l / d nu from the library (FP64 central difference, relative step
    1e-4) against the oracle's trace formula with the integral form of
    d K_nu / d nu, within 1e-6 of the scale sum_i |d l_i / d nu|; a plan
    taking two thetas per launch gives the same value as two launches."""
    from paper_2410_04477_amd import api
    th = W.Theta(1.2, 0.08, 1e-3, nu)
    pb = problem("gnu-dnu", 600, 2, 40, 30, W.Theta(1.2, 0.08, 1e-3, 1.5), 97)
    args = (pb["locs_perm"], pb["y_perm"], pb["block_ptr"], pb["nbr_ptr"], pb["nbr_idx"])
    ref = OL.grad_nu_trace(*args, th)
    lp, yp, nid = _t(pb["locs_perm"]), _t(pb["y_perm"]), _t(pb["nbr_idx"], torch.int32)
    bp, npt = _t(pb["block_ptr"], torch.int32), _t(pb["nbr_ptr"], torch.int32)
    got1 = float(api.loglik_dnu(api.Plan(bp, npt, 600, 1), lp, yp, nid, [th])[0])
    got2 = api.loglik_dnu(api.Plan(bp, npt, 600, 2), lp, yp, nid, [th, th.replace(nu=nu * 1.1)]).cpu().numpy()
    scale = np.abs(ref).sum()
    print(f"nu={nu}: dl/dnu gpu {got1:.9f} oracle {ref.sum():.9f} rel-to-scale {abs(got1 - ref.sum()) / scale:.1e}")
    assert abs(got1 - ref.sum()) <= 1e-6 * scale
    assert got2[0] == got1
    ref_b = OL.grad_nu_trace(*args, th.replace(nu=nu * 1.1))
    assert abs(got2[1] - ref_b.sum()) <= 1e-6 * np.abs(ref_b).sum()


def test_nu_derivative_error_paths():
    from paper_2410_04477_amd import api
    from paper_2410_04477_amd._lib import VecchiaError
    th = W.Theta(1.0, 0.1, 1e-3, 1.5)
    pb = problem("gnu-err", 400, 2, 40, 20, th, 91)
    lp, yp, nid = _t(pb["locs_perm"]), _t(pb["y_perm"]), _t(pb["nbr_idx"], torch.int32)
    bp, npt = _t(pb["block_ptr"], torch.int32), _t(pb["nbr_ptr"], torch.int32)
    plan = api.Plan(bp, npt, 400, 1)
    for step in (0.0, -1e-4, 0.5, float("nan")):
        with pytest.raises(VecchiaError, match="invalid"):
            api.loglik_dnu(plan, lp, yp, nid, [th], step)
    for nu, word in ((12.0, "unsupported"), (0.01, "unsupported"), (-1.0, "invalid")):
        with pytest.raises(VecchiaError, match=word):
            api.loglik_dnu(plan, lp, yp, nid, [th.replace(nu=nu)])
    with pytest.raises(VecchiaError, match="unsupported"):
        api.loglik_dnu(api.Plan(bp, npt, 400, 1, "tiles"), lp, yp, nid, [th])
    # at the edge of the range the stencil is one-sided and still finite
    d = api.loglik_dnu(plan, lp, yp, nid, [th.replace(nu=10.0)])
    assert torch.isfinite(d).all()


def test_mle_estimates_nu():
    """L-BFGS over (sigma2, range, nugget, nu) on a draw with nu = 1.5, started
    at nu = 0.8: the joint fit is at least as likely as the truth and as the
    fit with nu held at its start, and nu moves toward the truth."""
    from paper_2410_04477_amd import mle
    from paper_2410_04477_amd.model import BlockVecchia
    th = W.Theta(1.0, 0.08, 0.01, 1.5)
    pb = problem("gnu-mle-nu", 2000, 2, 200, 30, th, 87)
    mod = BlockVecchia.from_prepared(_t(pb["locs_perm"]), _t(pb["y_perm"]), _t(pb["block_ptr"], torch.int32),
                                     _t(pb["nbr_ptr"], torch.int32), _t(pb["nbr_idx"], torch.int32), 0.8)
    joint = mle.fit(mod, (1.0, 0.05, 0.05, 0.8), "fp64", max_evals=120, estimate_nu=True)
    fixed = mle.fit(mod, (1.0, 0.05, 0.05), "fp64", max_evals=120)
    ll_true = float(mod.loglik([mod.theta(th.sigma2, th.beta, th.nugget, th.nu)])[0][0])
    print("joint", joint.theta, joint.loglik, joint.evals, "fixed nu=0.8", fixed.theta, fixed.loglik,
          "truth", ll_true)
    assert len(joint.theta) == 4
    assert joint.loglik >= ll_true - 1e-6 * abs(ll_true)
    assert joint.loglik >= fixed.loglik - 1e-6 * abs(fixed.loglik)
    assert abs(joint.theta[3] - 1.5) < abs(0.8 - 1.5)


def test_nu_derivative_3d_anisotropic():
    """d l / d nu on a 3-D anisotropic problem (range a common scale,
    multipliers (1, 1, 0.2)) against the oracle's trace formula."""
    from paper_2410_04477_amd import api
    th = W.Theta(1.0, 0.1, 1e-3, 1.8, (1.0, 1.0, 0.2))
    pb = problem("gnu-dnu-3d", 500, 3, 40, 25, th.replace(nu=1.5), 99, zmax=0.2)
    args = (pb["locs_perm"], pb["y_perm"], pb["block_ptr"], pb["nbr_ptr"], pb["nbr_idx"])
    ref = OL.grad_nu_trace(*args, th)
    plan = api.Plan(_t(pb["block_ptr"], torch.int32), _t(pb["nbr_ptr"], torch.int32), 500, 1)
    got = float(api.loglik_dnu(plan, _t(pb["locs_perm"]), _t(pb["y_perm"]), _t(pb["nbr_idx"], torch.int32), [th])[0])
    print(f"3-D: dl/dnu gpu {got:.9f} oracle {ref.sum():.9f}")
    assert abs(got - ref.sum()) <= 1e-6 * np.abs(ref).sum()


def test_mle_estimates_nu_fp32_bulk():
    """The joint fit with the FP32-bulk gradient (then the FP64 polish) reaches
    the FP64 joint fit's likelihood."""
    from paper_2410_04477_amd import mle
    from paper_2410_04477_amd.model import BlockVecchia
    th = W.Theta(1.0, 0.08, 0.01, 1.5)
    pb = problem("gnu-mle-nu", 2000, 2, 200, 30, th, 87)
    mod = BlockVecchia.from_prepared(_t(pb["locs_perm"]), _t(pb["y_perm"]), _t(pb["block_ptr"], torch.int32),
                                     _t(pb["nbr_ptr"], torch.int32), _t(pb["nbr_idx"], torch.int32), 0.8)
    r64 = mle.fit(mod, (1.0, 0.05, 0.05, 0.8), "fp64", max_evals=120, estimate_nu=True)
    r32 = mle.fit(mod, (1.0, 0.05, 0.05, 0.8), "fp32", max_evals=120, estimate_nu=True)
    print("fp64", r64.theta, r64.loglik, "fp32-bulk + polish", r32.theta, r32.loglik)
    assert r32.loglik >= r64.loglik - 1e-6 * abs(r64.loglik)


@pytest.mark.parametrize("nu,d", [(0.5, 2), (1.3, 2), (1.5, 2), (3.7, 2), (1.8, 3)])
def test_adjoint_nu_gradient_matches_oracle_per_block(nu, d):
    """vecchia_loglik_grad_nu: d l_i / d nu from the adjoint (d K_nu / d nu by
    quadrature in the contraction) per block against the oracle's trace
    formula, within 1e-8 of each row's scale (FP64), and the other three
    components equal to vecchia_loglik_grad's to rounding; FP32-bulk within
    1e-3 norm-wise; the total agrees with the FP64 central difference in nu.
    The half-integers go through the Bessel-form kernels too."""
    from paper_2410_04477_amd import api
    aniso = (1.0, 1.0, 0.2) if d == 3 else (1.0, 1.0, 1.0)
    th = W.Theta(1.2, 0.08, 1e-3, nu, aniso)
    pb = problem(f"gnu-adj-{d}", 700, d, 50, 30, W.Theta(1.2, 0.08, 1e-3, 1.5, aniso), 95 + d,
                 zmax=0.2 if d == 3 else 1.0)
    args = (pb["locs_perm"], pb["y_perm"], pb["block_ptr"], pb["nbr_ptr"], pb["nbr_idx"])
    ref = OL.grad_nu_trace(*args, th)
    lp, yp, nid = _t(pb["locs_perm"]), _t(pb["y_perm"]), _t(pb["nbr_idx"], torch.int32)
    bp, npt = _t(pb["block_ptr"], torch.int32), _t(pb["nbr_ptr"], torch.int32)
    plan = api.Plan(bp, npt, 700, 1)
    ll, g4, cnt, part, gp4 = api.loglik_grad_nu(plan, lp, yp, nid, [th], "fp64", want_partial=True)
    rows = gp4[0, :, 3].cpu().numpy()
    scale = np.abs(ref).max()
    print(f"nu={nu} d={d}: dl/dnu adjoint {float(g4[0, 3]):.10f} oracle {ref.sum():.10f}; "
          f"max row err / max |row| {np.abs(rows - ref).max() / scale:.1e}", flush=True)
    np.testing.assert_allclose(rows, ref, rtol=1e-8, atol=1e-8 * scale)
    l3, g3, _, p3, gp3 = api.loglik_grad(plan, lp, yp, nid, [th], "fp64", want_partial=True)
    np.testing.assert_allclose(gp4[0, :, :3].cpu().numpy(), gp3[0].cpu().numpy(), rtol=1e-9,
                               atol=1e-10 * float(gp3.abs().max()))
    assert abs(float(ll[0]) - float(l3[0])) <= 1e-10 * abs(float(l3[0]))
    fd = float(api.loglik_dnu(plan, lp, yp, nid, [th])[0])
    assert abs(float(g4[0, 3]) - fd) <= 1e-6 * np.abs(ref).sum()
    _, g32, _, _, gp32 = api.loglik_grad_nu(plan, lp, yp, nid, [th], "fp32", want_partial=True)
    r32 = gp32[0, :, 3].cpu().numpy()
    assert np.linalg.norm(r32 - ref) <= 1e-3 * np.linalg.norm(ref)


def test_adjoint_nu_gradient_rejects_other_engines():
    from paper_2410_04477_amd import api
    from paper_2410_04477_amd._lib import VecchiaError
    th = W.Theta(1.0, 0.1, 1e-3, 1.3)
    pb = problem("gnu-err", 400, 2, 40, 20, W.Theta(1.0, 0.1, 1e-3, 1.5), 91)
    lp, yp, nid = _t(pb["locs_perm"]), _t(pb["y_perm"]), _t(pb["nbr_idx"], torch.int32)
    bp, npt = _t(pb["block_ptr"], torch.int32), _t(pb["nbr_ptr"], torch.int32)
    for eng in ("tiles", "mfma_wg"):
        with pytest.raises(VecchiaError, match="unsupported"):
            api.loglik_grad_nu(api.Plan(bp, npt, 400, 1, eng), lp, yp, nid, [th])
