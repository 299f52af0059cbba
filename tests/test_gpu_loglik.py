"""GPU parity of the fused block kernels against the FP64 oracle, on identical
oracle-produced inputs, through the C ABI.

Tolerances: FP64 path <= 1e-8 relative on the total log-likelihood (per
block <= 1e-8 relative + 1e-9 absolute); FP32-bulk path <= 1e-4 relative on
the total."""
import numpy as np
import pytest
import torch

import workloads as W
from cases import oracle_sum, oracle_terms, problem, workload_problem
from oracle import loglik as OL

pytestmark = pytest.mark.gpu
# one-wave matrix-core (default), four-wave matrix-core, vector-ALU register tiles
ENGINES = ["mfma", "mfma_wg", "tiles"]

DEV = "cuda"


def _gpu(pb, thetas, precision="fp64", max_theta=None, engine="mfma"):
    from paper_2410_04477_amd import api
    lp = torch.tensor(pb["locs_perm"], device=DEV)
    yp = torch.tensor(pb["y_perm"], device=DEV)
    bp = torch.tensor(pb["block_ptr"], dtype=torch.int32, device=DEV)
    npt = torch.tensor(pb["nbr_ptr"], dtype=torch.int32, device=DEV)
    nidx = torch.tensor(pb["nbr_idx"] if len(pb["nbr_idx"]) else [0], dtype=torch.int32, device=DEV)
    plan = api.Plan(bp, npt, pb["n"], max_theta or len(thetas), engine)
    ll, cnt, part = api.loglik(plan, lp, yp, nidx, thetas, precision, want_partial=True)
    torch.cuda.synchronize()
    return ll.cpu().numpy(), cnt.cpu().numpy(), part.cpu().numpy(), plan


def _check_fp64(pb, thetas, engine="mfma"):
    ll, cnt, part, _ = _gpu(pb, thetas, "fp64", engine=engine)
    for t, th in enumerate(thetas):
        ref_terms = oracle_terms(pb, th)
        ref = oracle_sum(ref_terms)
        np.testing.assert_allclose(part[t], ref_terms, rtol=1e-8, atol=1e-9)
        assert abs(ll[t] - ref) <= 1e-8 * abs(ref), (t, ll[t], ref)
        assert cnt[t, 1] == 0
    return ll


def test_fp64_c1_all_grid_thetas():
    w = W.C1
    pb = workload_problem(w, ysim="exact")
    thetas = W.theta_grid_c1()
    ll = _check_fp64(pb, thetas)
    worst = max(abs(ll[t] - oracle_sum(oracle_terms(pb, th))) / abs(oracle_sum(oracle_terms(pb, th)))
                for t, th in enumerate(thetas))
    print(f"C1 worst rel err fp64 {worst:.2e} over {len(thetas)} thetas")


@pytest.mark.parametrize("engine", ENGINES)
def test_fp32_bulk_c1_grid(engine):
    w = W.C1
    pb = workload_problem(w, ysim="exact")
    thetas = W.theta_grid_c1()
    ll, cnt, _, _ = _gpu(pb, thetas, "fp32", engine=engine)
    worst = 0.0
    for t, th in enumerate(thetas):
        ref = oracle_sum(oracle_terms(pb, th))
        worst = max(worst, abs(ll[t] - ref) / abs(ref))
        assert abs(ll[t] - ref) <= 1e-4 * abs(ref), (t, ll[t], ref, cnt[t])
    print(f"C1 worst rel err fp32-bulk ({engine}) {worst:.2e}; refactored {int(cnt[:, 0].sum())} of "
          f"{len(thetas) * (pb['block_ptr'].size - 1)}")


@pytest.mark.parametrize("nu,d", [(0.5, 2), (1.5, 2), (2.5, 3)])
def test_all_previous_conditioning_equals_exact_gp(nu, d):
    th = W.Theta(1.0, 0.1, 1e-4, nu, (1.0, 1.0, 0.5) if d == 3 else (1.0, 1.0, 1.0))
    pb = problem(f"exact{nu}", 160, d, 16, -1, th, 11)
    ll, cnt, _, _ = _gpu(pb, [th])
    ex = OL.exact_loglik(pb["locs_perm"], pb["y_perm"], th)
    assert abs(ll[0] - ex) <= 1e-9 * abs(ex)


def test_block_size_one_is_classic_vecchia():
    th = W.Theta(1.3, 0.08, 1e-3, 1.5)
    n, m = 400, 25
    g = W.rng(21)
    s = g.random((n, 2))
    from oracle import preprocess as P, simulate as S
    order = W.point_permutation(n, 21)
    so = s[order]
    bp = np.arange(n + 1)
    nptr, nidx = P.block_neighbors(so, bp, [1.0, 1.0], m)
    yo = S.exact_gp(so, th, W.standard_normal(n, 22))
    pb = dict(locs_perm=so, y_perm=yo, block_ptr=bp, nbr_ptr=nptr, nbr_idx=nidx, n=n, d=2)
    ll, _, _, _ = _gpu(pb, [th])
    cv = OL.classic_vecchia_loglik(so, yo, [nidx[nptr[i]:nptr[i + 1]] for i in range(n)], th)
    assert abs(ll[0] - cv) <= 1e-9 * abs(cv)


@pytest.mark.parametrize("m,bc", [(0, 100), (4, 100), (9, 100), (17, 100), (27, 100), (38, 100), (44, 100),
                                  (55, 100), (66, 100), (84, 100), (103, 100), (125, 100), (139, 100),
                                  (150, 250), (163, 500)])
@pytest.mark.parametrize("engine", ENGINES)
def test_every_tile_configuration_ragged(m, bc, engine):
    """m sweeps the joint size across every register-tile configuration and
    its ragged tail (p not a multiple of the tile size)."""
    th = W.Theta(0.9, 0.07, 5e-4, 2.5, (1.0, 1.0, 0.3))
    pb = problem(f"rag{m}", 1500, 3, bc, m, th, 31 + m, zmax=0.3)
    assert (np.diff(pb["block_ptr"]) + np.diff(pb["nbr_ptr"])).max() <= 175
    _check_fp64(pb, [th, th.replace(nu=0.5, beta=0.05), th.replace(nu=1.5, sigma2=2.0)], engine)


@pytest.mark.parametrize("engine", ENGINES)
def test_joint_size_above_register_capacity(engine):
    """m_i + l_i > 175 goes to the global-workspace panel kernel."""
    th = W.Theta(1.0, 0.1, 1e-3, 1.5)
    pb = problem("large", 3000, 2, 150, 200, th, 3, ysim="block")
    assert (np.diff(pb["block_ptr"]) + np.diff(pb["nbr_ptr"])).max() > 175
    _check_fp64(pb, [th, th.replace(nu=2.5)], engine)
    ll32, cnt, _, _ = _gpu(pb, [th], "fp32", engine=engine)
    ref = oracle_sum(oracle_terms(pb, th))
    assert abs(ll32[0] - ref) <= 1e-4 * abs(ref)


def test_exact_gp_n2000_all_previous_conditioning():
    """Every block conditions on all earlier points (p up to 2,000): the block
    Vecchia value equals the exact GP log-likelihood, for every grid theta."""
    w = W.C1
    s = W.locations(w)
    from oracle import preprocess as P, simulate as S
    lab, _ = P.kmeans(s, w.metric_scale, W.kmeans_init(w.n, w.bc, w.seed_kmeans), 30)
    perm, bp = P.order_blocks(lab, W.block_permutation(w.bc, w.seed_kmeans))
    lp = s[perm]
    nptr, nidx = P.block_neighbors(lp, bp, w.metric_scale, -1)
    yp = S.exact_gp(lp, w.theta, W.standard_normal(w.n, w.seed_y))
    pb = dict(locs_perm=lp, y_perm=yp, block_ptr=bp, nbr_ptr=nptr, nbr_idx=nidx, n=w.n, d=2)
    thetas = W.theta_grid_c1()
    ll, cnt, _, plan = _gpu(pb, thetas, "fp64")
    assert plan.c.nlarge > 0
    for t, th in enumerate(thetas):
        ex = OL.exact_loglik(lp, yp, th)
        assert abs(ll[t] - ex) <= 1e-10 * abs(ex), (t, ll[t], ex)


@pytest.mark.parametrize("engine", ENGINES)
def test_fp32_forced_refactor_reproduces_fp64(engine):
    th = W.Theta(1.0, 0.05, 1e-4, 1.5)
    pb = problem("force", 3000, 2, 300, 40, th, 41, ysim="block")
    ll64, _, p64, _ = _gpu(pb, [th], "fp64", engine=engine)
    llf, cnt, pf, _ = _gpu(pb, [th], "fp32_force_refactor", engine=engine)
    assert cnt[0, 0] == 300 and cnt[0, 1] == 0
    np.testing.assert_array_equal(pf, p64)
    assert llf[0] == ll64[0]


def test_non_pd_block_reports_nan_and_counter():
    th = W.Theta(1.0, 0.1, 0.0, 0.5)
    s = W.rng(5).random((50, 2))
    s[7] = s[3]  # duplicate location, zero nugget: singular covariance
    pb = dict(locs_perm=s, y_perm=W.standard_normal(50, 1), block_ptr=np.array([0, 5, 12, 50]),
              nbr_ptr=np.array([0, 0, 5, 15]), nbr_idx=np.concatenate([np.arange(5), np.arange(10)]), n=50, d=2)
    ll, cnt, _, _ = _gpu(pb, [th], "fp64")
    assert np.isnan(ll[0]) and cnt[0, 1] >= 1


def test_c2_full_size_fp64_and_fp32_grid():
    """n = 100,000, 10,000 blocks, m = 60, all 50 grid thetas in one call."""
    w = W.C2
    pb = workload_problem(w, ysim="block")
    thetas = W.theta_grid_c2()
    ll64, c64, _, _ = _gpu(pb, thetas, "fp64")
    ll32, c32, _, _ = _gpu(pb, thetas, "fp32")
    ll32t, _, _, _ = _gpu(pb, thetas, "fp32", engine="tiles")
    worst64 = worst32 = 0.0
    for t, th in enumerate(thetas):
        ref = oracle_sum(oracle_terms(pb, th))
        worst64 = max(worst64, abs(ll64[t] - ref) / abs(ref))
        worst32 = max(worst32, abs(ll32[t] - ref) / abs(ref), abs(ll32t[t] - ref) / abs(ref))
    print(f"C2 worst rel err fp64 {worst64:.2e} fp32 {worst32:.2e}; refactored {c32[:, 0].sum()}")
    assert worst64 <= 1e-8
    assert worst32 <= 1e-4
