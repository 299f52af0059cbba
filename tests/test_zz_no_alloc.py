"""vecchia_loglik_noalloc (the value path with its per-call buffers in the
library's static device array) against vecchia_loglik, called through the C
ABI: two calls in a row on different plans, the second on a smaller input,
each compared element by element with the workspace entry point."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W
from oracle import preprocess as P, simulate as S

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _t(a, dt=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device=DEV)


def _problem(n, bc, m, seed, th):
    g = W.rng(seed)
    s = g.random((n, 2))
    lab, _ = P.kmeans(s, [1.0, 1.0], W.kmeans_init(n, bc, seed), 30)
    perm, bp = P.order_blocks(lab, W.block_permutation(bc, seed))
    lp = s[perm]
    nptr, nidx = P.block_neighbors(lp, bp, [1.0, 1.0], m)
    yp = S.exact_gp(lp, th, W.standard_normal(n, seed + 1))
    return lp, yp, bp, nptr, nidx


def _call(fn, plan, lp, yp, nid, thetas, prec):
    from paper_2410_04477_amd import _lib as L
    from paper_2410_04477_amd.api import _p, _stream, make_theta
    th = [make_theta(t) for t in thetas]
    arr = (L.Theta * len(th))(*th)
    out = torch.full((len(th),), float("nan"), dtype=torch.float64, device=DEV)
    cnt = torch.full((len(th), 2), -1, dtype=torch.int32, device=DEV)
    part = torch.full((len(th), plan.bc), float("nan"), dtype=torch.float64, device=DEV)
    st = fn(ctypes.byref(plan.c), _p(lp), _p(yp), 2, _p(plan.block_ptr), _p(plan.nbr_ptr), _p(nid), arr, len(th),
            {"fp64": L.FP64, "fp32": L.FP32_BULK, "force": 2}[prec], _p(out), _p(cnt), _p(part), _stream())
    torch.cuda.synchronize()
    return st, out.cpu().numpy(), cnt.cpu().numpy(), part.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "force"])
def test_noalloc_matches_workspace_entry_point(prec):
    from paper_2410_04477_amd import _lib as L, api
    lib = L.lib()
    assert lib.vecchia_noalloc_scratch_bytes() >= 16 * L.NOALLOC_MAX_ITEMS
    th = W.Theta(1.3, 0.07, 2e-3, 1.5)
    cases = [(6000, 500, 60, 3, 5), (1500, 120, 30, 1, 6)]   # (n, bc, m, ntheta, seed): second call smaller
    for n, bc, m, nt, seed in cases:
        print(f"noalloc {prec}: n={n} bc={bc} m={m} ntheta={nt}", flush=True)
        lp, yp, bp, nptr, nidx = _problem(n, bc, m, seed, th)
        thetas = [W.Theta(th.sigma2 * (1 + 0.1 * k), th.beta * (1 - 0.05 * k), th.nugget, th.nu) for k in range(nt)]
        plan = api.Plan(_t(bp, torch.int32), _t(nptr, torch.int32), n, nt)
        args = (plan, _t(lp), _t(yp), _t(nidx, torch.int32), thetas, prec)
        st0, ll0, c0, p0 = _call(lib.vecchia_loglik, *args)
        st1, ll1, c1, p1 = _call(lib.vecchia_loglik_noalloc, *args)
        assert st0 == L.OK and st1 == L.OK
        np.testing.assert_array_equal(ll1, ll0)
        np.testing.assert_array_equal(c1, c0)
        np.testing.assert_array_equal(p1, p0)
        assert np.all(np.isfinite(ll1))
        if prec == "force":
            assert np.all(c1[:, 0] == bc)


def test_noalloc_rejects_sizes_beyond_its_array():
    from paper_2410_04477_amd import _lib as L, api
    lib = L.lib()
    n, bc = 1200, 300
    lp, yp, bp, nptr, nidx = _problem(n, bc, 20, 9, W.Theta(1.0, 0.1, 1e-3, 0.5))
    nt = L.NOALLOC_MAX_ITEMS // bc + 1   # bc * nt just above the array's capacity
    plan = api.Plan(_t(bp, torch.int32), _t(nptr, torch.int32), n, nt, aux_bytes=1 << 22)
    thetas = [W.Theta(1.0, 0.1, 1e-3, 0.5)] * nt
    st, ll, _, _ = _call(lib.vecchia_loglik_noalloc, plan, _t(lp), _t(yp), _t(nidx, torch.int32), thetas, "fp64")
    assert st == L.ENOMEM
    assert np.all(np.isnan(ll))   # nothing was launched
    st, ll, _, _ = _call(lib.vecchia_loglik_noalloc, plan, _t(lp), _t(yp), _t(nidx, torch.int32), thetas[:3], "fp64")
    assert st == L.OK and np.all(np.isfinite(ll))
