"""Edge cases and error paths of the C ABI on the GPU: invalid and unsupported
parameters, capacity limits, degenerate block structures.  Errors must come
back as status codes (VecchiaError in the binding), never as wrong values."""
import numpy as np
import pytest
import torch

import workloads as W
from cases import oracle_sum, oracle_terms, problem
from oracle import loglik as OL

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _tensors(pb):
    t = lambda a, dt: torch.tensor(np.asarray(a), dtype=dt, device=DEV)
    nidx = pb["nbr_idx"] if len(pb["nbr_idx"]) else np.zeros(1)
    return (t(pb["locs_perm"], torch.float64), t(pb["y_perm"], torch.float64),
            t(pb["block_ptr"], torch.int32), t(pb["nbr_ptr"], torch.int32), t(nidx, torch.int32))


def _plan(pb, max_theta=1, engine="mfma"):
    from paper_2410_04477_amd import api
    lp, yp, bp, npt, nidx = _tensors(pb)
    return api.Plan(bp, npt, pb["n"], max_theta, engine), lp, yp, nidx


def test_invalid_and_unsupported_theta_are_status_codes():
    from paper_2410_04477_amd import api
    from paper_2410_04477_amd._lib import VecchiaError
    th = W.Theta(1.0, 0.1, 1e-3, 1.5)
    pb = problem("edge", 400, 2, 40, 20, th, 91)
    plan, lp, yp, nidx = _plan(pb, max_theta=2)
    good = (1.0, 0.1, 1e-3, 1.5)
    for bad, word in (((0.0, 0.1, 1e-3, 1.5), "invalid"), ((1.0, -0.1, 1e-3, 1.5), "invalid"),
                      ((1.0, 0.1, -1e-3, 1.5), "invalid"), ((float("nan"), 0.1, 1e-3, 1.5), "invalid"),
                      ((1.0, 0.1, 1e-3, 12.0), "unsupported"), ((1.0, 0.1, 1e-3, 0.5, (1.0, 0.0, 1.0)), "invalid")):
        with pytest.raises(VecchiaError, match=word):
            api.loglik(plan, lp, yp, nidx, [good, bad])
        with pytest.raises(VecchiaError, match=word):
            api.loglik_grad(plan, lp, yp, nidx, [bad])
    # more thetas than the plan was built for
    with pytest.raises(VecchiaError, match="invalid"):
        api.loglik(plan, lp, yp, nidx, [good] * 3)
    # the valid call still works after the rejected ones
    ll, _, _ = api.loglik(plan, lp, yp, nidx, [good])
    ref = oracle_sum(oracle_terms(pb, th))
    assert abs(float(ll[0]) - ref) <= 1e-8 * abs(ref)


def test_empty_schedule_is_rejected():
    from paper_2410_04477_amd import api
    from paper_2410_04477_amd._lib import VecchiaError
    bp = torch.zeros(1, dtype=torch.int32, device=DEV)
    with pytest.raises(VecchiaError):
        api.Plan(bp, bp.clone(), 10, 1)


@pytest.mark.parametrize("engine", ["mfma", "mfma_wg", "tiles"])
def test_single_block_is_exact_gp(engine):
    """One block holding every point (m = 0, p = n = 150): the value is the
    exact GP log-likelihood, and the gradient matches the oracle."""
    from paper_2410_04477_amd import api
    th = W.Theta(1.3, 0.2, 5e-3, 2.5)
    pb = problem("one", 150, 2, 1, 0, th, 92)
    assert len(pb["block_ptr"]) == 2
    plan, lp, yp, nidx = _plan(pb, engine=engine)
    ll, cnt, _ = api.loglik(plan, lp, yp, nidx, [th])
    ex = OL.exact_loglik(pb["locs_perm"], pb["y_perm"], th)
    assert abs(float(ll[0]) - ex) <= 1e-9 * abs(ex)
    from oracle import coracle
    from paper_2410_04477_amd._lib import VecchiaError
    try:
        _, g, _, _, _ = api.loglik_grad(plan, lp, yp, nidx, [th])
    except VecchiaError as e:   # engines that hold all 152 right-hand sides in LDS
        assert engine != "mfma" and "unsupported" in str(e)
        return
    ref = coracle.grad_terms(pb["locs_perm"], pb["y_perm"], pb["block_ptr"], pb["nbr_ptr"], pb["nbr_idx"], th).sum(0)
    assert np.linalg.norm(g[0].cpu().numpy() - ref) <= 1e-8 * np.linalg.norm(ref)


def test_gradient_of_plans_with_large_blocks_is_unsupported():
    from paper_2410_04477_amd import api
    from paper_2410_04477_amd._lib import VecchiaError
    th = W.Theta(1.0, 0.1, 1e-3, 1.5)
    pb = problem("large-g", 1200, 2, 40, 190, th, 93)
    assert (np.diff(pb["block_ptr"]) + np.diff(pb["nbr_ptr"])).max() > 175
    plan, lp, yp, nidx = _plan(pb)
    assert plan.c.nlarge > 0
    with pytest.raises(VecchiaError, match="unsupported"):
        api.loglik_grad(plan, lp, yp, nidx, [th])
    ll, _, _ = api.loglik(plan, lp, yp, nidx, [th])
    ref = oracle_sum(oracle_terms(pb, th))
    assert abs(float(ll[0]) - ref) <= 1e-8 * abs(ref)


def test_many_thetas_cross_launch_batches():
    """More thetas than one launch carries (24): batches of the theta loop."""
    from paper_2410_04477_amd import api
    th = W.Theta(1.0, 0.08, 2e-3, 0.5)
    pb = problem("batch", 600, 2, 60, 25, th, 94)
    thetas = [th.replace(beta=0.03 + 0.004 * k, sigma2=0.8 + 0.01 * k) for k in range(53)]
    plan, lp, yp, nidx = _plan(pb, max_theta=len(thetas))
    ll, _, _ = api.loglik(plan, lp, yp, nidx, thetas)
    llg, g, _, _, _ = api.loglik_grad(plan, lp, yp, nidx, thetas, "fp64")
    for k in (0, 23, 24, 47, 52):
        ref = oracle_sum(oracle_terms(pb, thetas[k]))
        assert abs(float(ll[k]) - ref) <= 1e-8 * abs(ref)
        assert abs(float(llg[k]) - ref) <= 1e-8 * abs(ref)
