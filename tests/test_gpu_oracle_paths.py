"""Paths of the library that ordinary inputs do not reach, judged by the
oracle: the FP32 guard tripped by the data themselves (near-duplicate
points and a tiny nugget), the adjoint launched in chunks of a small factor
tile buffer, K-means clusters that start empty, and the rejection of a block
permutation that is not one."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import coracle, matern, preprocess as P, simulate as S

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _t(a, dt=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device=DEV)


def _near_duplicate_problem(n=4000, bc=400, m=30, frac=0.003, off=5e-5, seed=77):
    """Uniform points in the unit square where a fraction of them is moved to
    within `off` of another point.  With nu = 1.5, range 0.05 and nugget 1e-6
    the conditional variance of such a point given its twin is ~(off/range)^2
    + 2 nugget ~ 3e-6: positive definite in FP64 (smallest eigenvalue >= the
    nugget), but in FP32 the pivot drowns in rounding of order p 2^-24 and
    falls under the guard max(nugget / 2, p 2^-23 (sigma2 + nugget))."""
    th = W.Theta(1.0, 0.05, 1e-6, 1.5)
    g = W.rng(seed)
    s = g.random((n, 2))
    k = max(1, int(frac * n))
    src = g.choice(n, k, replace=False)
    dst = g.choice(np.setdiff1d(np.arange(n), src), k, replace=False)
    ang = g.uniform(0.0, 2.0 * np.pi, k)
    s[dst] = s[src] + off * np.c_[np.cos(ang), np.sin(ang)]
    lab, _ = P.kmeans(s, [1.0, 1.0], W.kmeans_init(n, bc, seed), 30)
    perm, bp = P.order_blocks(lab, W.block_permutation(bc, seed))
    lp = s[perm]
    nptr, nidx = P.block_neighbors(lp, bp, [1.0, 1.0], m)
    yp = S.exact_gp(lp, th, W.standard_normal(n, seed + 1))
    return th, lp, yp, bp, nptr, nidx


def test_fp32_guard_trips_on_near_duplicate_points():
    from paper_2410_04477_amd import api
    th, lp, yp, bp, nptr, nidx = _near_duplicate_problem()
    bc = bp.size - 1
    ref_l = coracle.block_terms(lp, yp, bp, nptr, nidx, th)
    ref_g = coracle.grad_terms(lp, yp, bp, nptr, nidx, th)
    assert np.all(np.isfinite(ref_l))
    ref_tot = float(np.sum(ref_l))
    lp_t, yp_t, bp_t, npt_t, nid_t = _t(lp), _t(yp), _t(bp, torch.int32), _t(nptr, torch.int32), _t(nidx, torch.int32)
    plan = api.Plan(bp_t, npt_t, lp.shape[0], 1)
    # FP64: every block within 1e-8 of the oracle
    ll64, _, part64 = api.loglik(plan, lp_t, yp_t, nid_t, [th], "fp64", want_partial=True)
    np.testing.assert_allclose(part64[0].cpu().numpy(), ref_l, rtol=1e-8, atol=1e-9)
    # FP32-bulk value: the guard flags some blocks, which are re-run in FP64
    ll, cnt, part = api.loglik(plan, lp_t, yp_t, nid_t, [th], "fp32", want_partial=True)
    flags = plan.flags()[0].cpu().numpy()
    refac = (flags & 4) != 0
    nref = int(cnt[0, 0])
    print(f"guard: {nref} of {bc} blocks re-factorised in FP64; failed {int(cnt[0, 1])}", flush=True)
    assert 0 < nref < bc
    assert refac.sum() == nref and np.all((flags[refac] & 1) != 0)
    assert int(cnt[0, 1]) == 0
    got = part[0].cpu().numpy()
    np.testing.assert_allclose(got[refac], ref_l[refac], rtol=1e-8, atol=1e-9)
    rel = abs(float(ll[0]) - ref_tot) / abs(ref_tot)
    print(f"FP32-bulk total vs oracle: rel {rel:.2e}", flush=True)
    assert rel <= 1e-4
    # gradient path: the blocks it flags are re-run (value and gradient) in FP64
    llg, grad, cntg, partg, gpartg = api.loglik_grad(plan, lp_t, yp_t, nid_t, [th], "fp32", want_partial=True)
    flags_g = plan.flags()[0].cpu().numpy()
    refg = (flags_g & 4) != 0
    assert 0 < refg.sum() < bc and refg.sum() == int(cntg[0, 0])
    gp = gpartg[0].cpu().numpy()
    np.testing.assert_allclose(gp[refg], ref_g[refg], rtol=1e-7, atol=1e-8 * np.abs(ref_g[refg]).max())
    np.testing.assert_allclose(partg[0].cpu().numpy()[refg], ref_l[refg], rtol=1e-8, atol=1e-9)
    assert abs(float(llg[0]) - ref_tot) <= 1e-4 * abs(ref_tot)


@pytest.mark.parametrize("m,prec,bc", [(40, "fp64", 60), (40, "fp32", 60), (120, "fp32", 150), (120, "fp64", 150)])
def test_chunked_adjoint_matches_oracle(m, prec, bc):
    """Right-hand sides in several passes, and a factor tile buffer that holds
    only three work items.  With m = 40 and 60 blocks (up to 78 points a
    block) every class keeps its factor in the registers and takes its l + 2
    right-hand sides in several passes; with m = 120 the classes reach G = 10
    or 11 and the ones whose gradient goes through the tile buffer (FP64 above
    G = 9 in one launch; FP32 at G = 11 as the factorisation + tile store
    launch and the adjoint launch) run their adjoint in many launches.  Per-block results
    equal the unchunked call's bit for bit and the oracle's within the FP64
    (1e-7 per row) or FP32-bulk (1e-3 norm-wise) bars."""
    from paper_2410_04477_amd import api
    th = W.Theta(1.1, 0.08, 2e-3, 1.5)
    n = 3000
    g = W.rng(91 + m)
    s = g.random((n, 2))
    lab, _ = P.kmeans(s, [1.0, 1.0], W.kmeans_init(n, bc, 91 + m), 30)
    perm, bp = P.order_blocks(lab, W.block_permutation(bc, 91 + m))
    lp = s[perm]
    nptr, nidx = P.block_neighbors(lp, bp, [1.0, 1.0], m)
    yp = S.exact_gp(lp, th, W.standard_normal(n, 92 + m))
    args = [_t(lp), _t(yp), _t(nidx, torch.int32)]
    bp_t, npt_t = _t(bp, torch.int32), _t(nptr, torch.int32)
    full = api.Plan(bp_t, npt_t, n, 1)
    nb = int(full.c.nbuckets)
    gs = [int(c) + 1 for c in full.c.bucket_cfg[:nb]]
    kernels = [full.class_kernel(q, prec, True) for q in range(nb)]
    tiles = [q for q in range(nb) if kernels[q].endswith((",1>", ",3>"))]
    print(f"m={m} {prec}: classes G {gs}, l max {list(full.c.bucket_lmax[:nb])}, kernels {kernels}", flush=True)
    if m == 40:
        # the register-resident adjoint in several passes (28 right-hand sides each)
        assert not tiles and all(",5>" in k for k in kernels)
        assert max(int(full.c.bucket_lmax[q]) for q in range(nb)) + 2 > 2 * 28
        plans = (("full", full),)
    else:
        assert max(gs) >= 10 and (bool(tiles) == (prec == "fp64" or 11 in gs))
        gmax = max(gs)
        # one work item's FP64 slot: G (G + 1) / 2 tiles of 16 x 16 doubles and the border row
        small_bytes = 3 * ((gmax * (gmax + 1) // 2 * 256 + 16 * gmax) * 8)
        assert small_bytes < int(full.c.aux_ws_bytes) / 8
        small = api.Plan(bp_t, npt_t, n, 1, aux_bytes=small_bytes)
        assert int(small.c.aux_ws_bytes) == small_bytes
        print(f"tile buffer {int(full.c.aux_ws_bytes)} -> {small_bytes} bytes", flush=True)
        plans = (("full", full), ("small", small)) if tiles else (("full", full),)
    res = {}
    for name, plan in plans:
        ll, gr, cnt, part, gpart = api.loglik_grad(plan, args[0], args[1], args[2], [th], prec, want_partial=True)
        res[name] = (ll.cpu().numpy(), gr.cpu().numpy(), part.cpu().numpy(), gpart.cpu().numpy())
    last = plans[-1][0]
    for a, b in zip(res["full"], res[last]):
        np.testing.assert_array_equal(a, b)
    ref_g = coracle.grad_terms(lp, yp, bp, nptr, nidx, th)
    ref_l = coracle.block_terms(lp, yp, bp, nptr, nidx, th)
    gp, pt = res[last][3][0], res[last][2][0]
    if prec == "fp64":
        np.testing.assert_allclose(gp, ref_g, rtol=1e-7, atol=1e-8 * np.abs(ref_g).max())
        np.testing.assert_allclose(pt, ref_l, rtol=1e-8, atol=1e-9)
    else:
        assert np.linalg.norm(gp - ref_g) <= 1e-3 * np.linalg.norm(ref_g)
        assert abs(float(res[last][0][0]) - ref_l.sum()) <= 1e-4 * abs(ref_l.sum())


@pytest.mark.parametrize("x,init,bperm,perm_ref,bp_ref", [
    # duplicate starts: cluster 1 is empty after the first assignment and takes
    # x = 10, the point farthest from the updated centroid 3.25
    ([0.0, 1.0, 2.0, 10.0], [0, 0], [0, 1], [0, 1, 2, 3], [0, 3, 4]),
    # clusters 1 and 2 start empty: they take x = 20, then x = 0 (squared
    # distances to the updated centroid 6.6: 43.56, 31.36, 21.16, 11.56, 179.56);
    # clusters end as {10}, {20}, {0, 1, 2}, placed in the order 2, 0, 1
    ([0.0, 1.0, 2.0, 10.0, 20.0], [0, 0, 0], [2, 0, 1], [0, 1, 2, 3, 4], [0, 3, 4, 5]),
])
def test_blocks_empty_cluster_reseed_as_oracle(x, init, bperm, perm_ref, bp_ref):
    from paper_2410_04477_amd import api
    xs = np.asarray(x)[:, None]
    lab, _ = P.kmeans(xs, [1.0], np.asarray(init), 30)
    operm, obp = P.order_blocks(lab, np.asarray(bperm))
    assert operm.tolist() == perm_ref and obp.tolist() == bp_ref   # the oracle's own hand example
    perm, bp, iters = api.blocks(_t(xs), len(init), _t(init, torch.int64), _t(bperm, torch.int64), [1.0],
                                 max_iter=30)
    assert perm.cpu().numpy().tolist() == perm_ref
    assert bp.cpu().numpy().tolist() == bp_ref


def test_blocks_rejects_a_block_perm_that_is_not_a_permutation():
    from paper_2410_04477_amd import api
    from paper_2410_04477_amd._lib import VecchiaError
    n, bc = 2000, 50
    s = _t(W.rng(3).random((n, 2)))
    init = _t(W.kmeans_init(n, bc, 3), torch.int64)
    good = W.block_permutation(bc, 3)
    dup = good.copy()
    dup[7] = dup[8]
    out = good.copy()
    out[0] = bc
    neg = good.copy()
    neg[5] = -1
    for bad in (dup, out, neg):
        with pytest.raises(VecchiaError, match="invalid argument"):
            api.blocks(s, bc, init, _t(bad, torch.int64), [1.0, 1.0], max_iter=2)
    # the library is still usable after the rejected calls
    perm, bp, _ = api.blocks(s, bc, init, _t(good, torch.int64), [1.0, 1.0], max_iter=2)
    assert sorted(perm.cpu().numpy().tolist()) == list(range(n))
