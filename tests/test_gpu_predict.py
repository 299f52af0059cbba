"""Block Vecchia prediction (Alg. 2) and conditional simulation on the GPU
against the oracle: neighbour sets bit for bit, conditional means, variances
and block covariances within FP64 rounding, PICP / MSPE of the simulated
intervals, plus edge cases and the paper's prediction setting."""
import functools

import numpy as np
import pytest
import torch

import workloads as W
from oracle import coracle, predict as PR, preprocess as P

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _t(a, dt=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device=DEV)


@functools.lru_cache(maxsize=None)
def _pred_problem(n_obs, n_new, d, bc, m, theta, seed):
    """Observations and new locations of one field (block Vecchia draw on the
    oracle's own blocks), the new locations clustered and ordered by the
    oracle, and the oracle's neighbour sets."""
    g = W.rng(seed)
    n = n_obs + n_new
    s = g.random((n, d))
    if d == 3:
        s[:, 2] *= 0.2
    wscale = [1.0 / a for a in theta.aniso[:d]]
    bcy = max(1, n // 10)
    labels, _ = P.kmeans(s, wscale, W.kmeans_init(n, bcy, seed + 1), 10)
    perm, bp = P.order_blocks(labels, W.block_permutation(bcy, seed + 1))
    lp = s[perm]
    nptr, nidx = P.block_neighbors(lp, bp, wscale, 40)
    yp = coracle.simulate(lp, bp, nptr, nidx, theta, W.standard_normal(n, seed + 2))
    split = W.rng(seed + 3).permutation(n)
    obs, new = split[:n_obs], split[n_obs:]
    s_obs, y_obs = lp[obs], yp[obs]
    s_new, y_new = lp[new], yp[new]
    labels, _ = P.kmeans(s_new, wscale, W.kmeans_init(n_new, bc, seed + 4))
    perm_new, bpn = P.order_blocks(labels, W.block_permutation(bc, seed + 4))
    s_new, y_new = s_new[perm_new], y_new[perm_new]
    npt, nid = PR.pred_neighbors(s_obs, s_new, bpn, wscale, m)
    return dict(s_obs=s_obs, y_obs=y_obs, s_new=s_new, y_new=y_new, block_ptr=bpn, nbr_ptr=npt, nbr_idx=nid,
                wscale=wscale, d=d)


def _gpu_predict(pb, theta, want_cov=True):
    from paper_2410_04477_amd import api
    bp, npt = _t(pb["block_ptr"], torch.int32), _t(pb["nbr_ptr"], torch.int32)
    nid = _t(pb["nbr_idx"] if len(pb["nbr_idx"]) else np.zeros(1), torch.int32)
    plan = api.Plan(bp, npt, pb["s_new"].shape[0], 1, "mfma", predict=True)
    mean, var, cov = api.predict(plan, _t(pb["s_obs"]), _t(pb["y_obs"]), _t(pb["s_new"]), nid, theta, want_cov)
    torch.cuda.synchronize()
    return plan, mean.cpu().numpy(), var.cpu().numpy(), None if cov is None else cov.cpu().numpy()


CASES = [  # (n_obs, n_new, d, bc, m, theta)
    (3000, 400, 2, 40, 30, W.Theta(1.0, 0.1, 1e-3, 0.5)),
    (4000, 600, 2, 60, 61, W.Theta(1.3, 0.07, 1e-3, 1.5)),
    (6000, 500, 3, 25, 120, W.Theta(1.0, 0.05, 1e-3, 2.5, (1.0, 1.0, 0.2))),
    (2500, 300, 2, 20, 130, W.Theta(0.8, 0.08, 1e-2, 2.5)),
    (1500, 200, 2, 20, 7, W.Theta(1.0, 0.2, 0.0, 1.5)),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_prediction_neighbours_match_oracle(case):
    from paper_2410_04477_amd import api
    n_obs, n_new, d, bc, m, th = CASES[case]
    pb = _pred_problem(n_obs, n_new, d, bc, m, th, 100 + case)
    npt, nid = api.pred_neighbors(_t(pb["s_obs"]), _t(pb["s_new"]), _t(pb["block_ptr"], torch.int32), m,
                                  pb["wscale"])
    assert np.array_equal(npt.cpu().numpy(), pb["nbr_ptr"])
    assert np.array_equal(nid.cpu().numpy(), pb["nbr_idx"])


@pytest.mark.parametrize("case", range(len(CASES)))
def test_prediction_matches_oracle(case):
    n_obs, n_new, d, bc, m, th = CASES[case]
    pb = _pred_problem(n_obs, n_new, d, bc, m, th, 100 + case)
    mean_o, var_o, covs_o = PR.predict(pb["s_obs"], pb["y_obs"], pb["s_new"], pb["block_ptr"], pb["nbr_ptr"],
                                       pb["nbr_idx"], th)
    plan, mean, var, cov = _gpu_predict(pb, th)
    gs = sorted({int(c) + 1 for c in plan.c.bucket_cfg[:plan.c.nbuckets]})
    print(f"case {case}: size classes G = {gs}")
    scale = th.sigma2 + th.nugget
    assert np.all(np.isfinite(mean)) and np.all(np.isfinite(var))
    assert np.max(np.abs(mean - mean_o)) <= 1e-8 * max(1.0, np.max(np.abs(mean_o)))
    assert np.max(np.abs(var - var_o)) <= 1e-9 * scale
    bp = pb["block_ptr"]
    for i in range(bp.size - 1):
        li = bp[i + 1] - bp[i]
        assert np.max(np.abs(cov[i, :li, :li] - covs_o[i])) <= 1e-9 * scale


def test_all_observations_is_exact_kriging_and_large_classes():
    """m = -1 with 150 observations: every block conditions on all of them
    (G up to 11 tile rows), which is exact kriging of the block."""
    from paper_2410_04477_amd import api
    th = W.Theta(1.1, 0.15, 5e-3, 2.5)
    g = W.rng(131)
    s_obs, s_new = g.random((150, 2)), g.random((60, 2))
    from oracle import simulate
    y_all = simulate.exact_gp(np.vstack([s_obs, s_new]), th, g.standard_normal(210))
    y_obs = y_all[:150]
    bp = np.array([0, 5, 17, 20, 21, 40, 60])
    npt, nid = PR.pred_neighbors(s_obs, s_new, bp, [1.0, 1.0], -1)
    gn, gi = api.pred_neighbors(_t(s_obs), _t(s_new), _t(bp, torch.int32), -1)
    assert np.array_equal(gn.cpu().numpy(), npt) and np.array_equal(gi.cpu().numpy(), nid)
    pb = dict(s_obs=s_obs, y_obs=y_obs, s_new=s_new, block_ptr=bp, nbr_ptr=npt, nbr_idx=nid)
    mean_o, var_o, covs_o = PR.predict(s_obs, y_obs, s_new, bp, npt, nid, th)
    plan, mean, var, cov = _gpu_predict(pb, th)
    assert max(int(c) + 1 for c in plan.c.bucket_cfg[:plan.c.nbuckets]) == 11
    assert np.max(np.abs(mean - mean_o)) <= 1e-7
    assert np.max(np.abs(var - var_o)) <= 1e-8
    for i in range(bp.size - 1):
        li = bp[i + 1] - bp[i]
        assert np.max(np.abs(cov[i, :li, :li] - covs_o[i])) <= 1e-8


def test_prediction_edge_cases():
    """No neighbours (the prior), one-point blocks, m above the number of
    observations, and the error paths."""
    from paper_2410_04477_amd import api
    from paper_2410_04477_amd._lib import VecchiaError
    th = W.Theta(1.4, 0.1, 0.02, 1.5)
    g = W.rng(141)
    s_obs, y_obs, s_new = g.random((9, 2)), g.standard_normal(9), g.random((7, 2))
    bp = np.array([0, 1, 4, 5, 7])
    for m in (0, 20):
        npt, nid = PR.pred_neighbors(s_obs, s_new, bp, [1.0, 1.0], m)
        gn, gi = api.pred_neighbors(_t(s_obs), _t(s_new), _t(bp, torch.int32), m)
        assert np.array_equal(gn.cpu().numpy(), npt) and np.array_equal(gi.cpu().numpy(), nid)
        pb = dict(s_obs=s_obs, y_obs=y_obs, s_new=s_new, block_ptr=bp, nbr_ptr=npt, nbr_idx=nid)
        mean_o, var_o, _ = PR.predict(s_obs, y_obs, s_new, bp, npt, nid, th)
        _, mean, var, _ = _gpu_predict(pb, th, want_cov=False)
        assert np.max(np.abs(mean - mean_o)) <= 1e-10
        assert np.max(np.abs(var - var_o)) <= 1e-10
        if m == 0:
            assert np.all(mean == 0.0) and np.allclose(var, th.sigma2 + th.nugget, rtol=1e-15)
    # a block too large for the one-wave kernel: pred_rows(m) + l > 175
    big = np.array([0, 7])
    npt = np.array([0, 170])
    with pytest.raises(VecchiaError, match="unsupported"):
        api.Plan(_t(big, torch.int32), _t(npt, torch.int32), 7, 1, "mfma", predict=True)
    # a prediction plan is not a likelihood plan, and needs one theta
    npt, nid = PR.pred_neighbors(s_obs, s_new, bp, [1.0, 1.0], 5)
    plan = api.Plan(_t(bp, torch.int32), _t(npt, torch.int32), 7, 1, "mfma", predict=True)
    with pytest.raises(VecchiaError, match="invalid"):
        api.loglik(plan, _t(s_new), _t(np.zeros(7)), _t(nid, torch.int32), [th])
    with pytest.raises(VecchiaError, match="invalid"):
        api.Plan(_t(bp, torch.int32), _t(npt, torch.int32), 7, 2, "mfma", predict=True)
    with pytest.raises(VecchiaError, match="unsupported"):
        api.predict(plan, _t(s_obs), _t(y_obs), _t(s_new), _t(nid, torch.int32), (1.0, 0.1, 0.0, 12.0))
    lplan = api.Plan(_t(bp, torch.int32), _t(npt, torch.int32), 7, 1, "mfma")
    with pytest.raises(VecchiaError, match="invalid"):
        api.predict(lplan, _t(s_obs), _t(y_obs), _t(s_new), _t(nid, torch.int32), th)


def test_condsim_matches_oracle():
    from paper_2410_04477_amd import api
    g = W.rng(151)
    n, r = 3001, 64
    mean = g.normal(size=n)
    var = g.uniform(0.1, 3.0, size=n)
    z = g.standard_normal((r, n))
    y = mean + np.sqrt(var) * g.standard_normal(n)
    ref = PR.condsim_stats(mean, var, z, y)
    out = api.condsim(_t(mean), _t(var), _t(z), _t(y))
    for k in ("sample_mean", "sample_sd", "lo", "hi"):
        assert np.max(np.abs(out[k].cpu().numpy() - ref[k])) <= 1e-12 * (1 + np.max(np.abs(ref[k]))), k
    # coverage is decided in FP64 on both sides: identical unless a truth sits
    # within rounding of an interval end
    lo, hi = ref["lo"], ref["hi"]
    amb = np.sum(np.minimum(np.abs(y - lo), np.abs(y - hi)) < 1e-12)
    assert abs(out["picp"] - ref["picp"]) <= amb / n
    assert out["mspe"] == pytest.approx(ref["mspe"], rel=1e-12)


def test_paper_prediction_setting_coverage():
    """The paper's prediction study: 20,000 points of one field, 90 % observed
    and 10 % held out, the held-out points in 200 blocks, true parameters, 1,000
    rounds of conditional simulation.  The GPU pipeline (its own K-means blocks,
    neighbours, prediction, simulation) gives about 95 % coverage, and on the
    oracle's blocks and neighbours the same PICP and MSPE as the oracle."""
    from paper_2410_04477_amd import api
    th = W.Theta(1.0, 0.1, 1e-3, 1.5)
    pb = _pred_problem(18000, 2000, 2, 200, 60, th, 161)
    z = W.rng(162).standard_normal((1000, 2000))
    mean_o, var_o, _ = PR.predict(pb["s_obs"], pb["y_obs"], pb["s_new"], pb["block_ptr"], pb["nbr_ptr"],
                                  pb["nbr_idx"], th)
    ref = PR.condsim_stats(mean_o, var_o, z, pb["y_new"])
    _, mean, var, _ = _gpu_predict(pb, th, want_cov=False)
    out = api.condsim(_t(mean), _t(var), _t(z), _t(pb["y_new"]))
    print(f"oracle PICP {ref['picp']:.4f} MSPE {ref['mspe']:.5f}; GPU PICP {out['picp']:.4f} MSPE {out['mspe']:.5f}")
    assert abs(out["picp"] - ref["picp"]) <= 1.0 / 2000
    assert out["mspe"] == pytest.approx(ref["mspe"], rel=1e-9)
    # the whole pipeline on the GPU, from K-means of the held-out points on
    s_new_orig = pb["s_new"]
    bc = 200
    perm, bpg, _ = api.blocks(_t(s_new_orig), bc, _t(W.kmeans_init(2000, bc, 163), torch.int64),
                              _t(W.block_permutation(bc, 163), torch.int64), pb["wscale"])
    s_new_g = api.permute_rows(_t(s_new_orig), perm)
    y_new_g = api.permute_rows(_t(pb["y_new"]), perm)
    npt, nid = api.pred_neighbors(_t(pb["s_obs"]), s_new_g, bpg, 60, pb["wscale"])
    plan = api.Plan(bpg, npt, 2000, 1, "mfma", predict=True)
    mean_g, var_g, _ = api.predict(plan, _t(pb["s_obs"]), _t(pb["y_obs"]), s_new_g, nid, th)
    full = api.condsim(mean_g, var_g, _t(z), y_new_g)
    print(f"GPU pipeline PICP {full['picp']:.4f} MSPE {full['mspe']:.5f}")
    assert 0.93 <= full["picp"] <= 0.97
    assert full["mspe"] == pytest.approx(float(var_g.mean()), rel=0.15)


def test_model_level_predict_and_ordering():
    """BlockVecchia with a maxmin block order gives the oracle's likelihood on
    the same blocks, and its predict() matches the oracle's prediction."""
    from paper_2410_04477_amd.model import BlockVecchia
    from oracle import loglik as OL, ordering as O
    th = W.Theta(1.0, 0.1, 1e-3, 1.5)
    g = W.rng(171)
    s = g.random((2000, 2))
    from oracle import simulate
    y = simulate.exact_gp(s, th, g.standard_normal(2000))
    bv = BlockVecchia(s, y, 100, 30, 1.5, W.kmeans_init(2000, 100, 3), W.block_permutation(100, 3),
                      ordering="maxmin")
    lp, yp = bv.locs_perm.cpu().numpy(), bv.y_perm.cpu().numpy()
    bp = bv.block_ptr.cpu().numpy()
    # the order is the oracle's maxmin order of these blocks' centroids
    cen = P.block_centroids(lp, bp, [1.0, 1.0])
    assert np.array_equal(O.maxmin_order(cen), np.arange(bp.size - 1))
    npt, nid = P.block_neighbors(lp, bp, [1.0, 1.0], 30)
    ref = OL.loglik(lp, yp, bp, npt, nid, th)
    ll, _, _ = bv.loglik([(1.0, 0.1, 1e-3, 1.5)])
    assert abs(float(ll[0]) - ref) <= 1e-8 * abs(ref)
    s_new = g.random((300, 2))
    mean, var, _, perm, bpn = bv.predict(s_new, 30, 25, (1.0, 0.1, 1e-3, 1.5), W.kmeans_init(300, 30, 4),
                                         W.block_permutation(30, 4))
    sn = s_new[perm.cpu().numpy()]
    bpn = bpn.cpu().numpy()
    pnp, pni = PR.pred_neighbors(lp, sn, bpn, [1.0, 1.0], 25)
    mo, vo, _ = PR.predict(lp, yp, sn, bpn, pnp, pni, th)
    assert np.max(np.abs(mean.cpu().numpy() - mo)) <= 1e-9
    assert np.max(np.abs(var.cpu().numpy() - vo)) <= 1e-10
