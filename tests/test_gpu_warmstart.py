"""Learned warm start on the GPU: variogram features, BF16 matrix-core GEMMs,
MLP forward/backward/Adam against the FP64 oracle (with the same BF16
operand rounding), training, and warm- vs cold-start MLE."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import learned as OLR

pytestmark = pytest.mark.gpu
DEV = "cuda"


def test_variogram_features_vs_oracle():
    from paper_2410_04477_amd import api
    k, nsets = 1500, 3
    g = W.rng(5)
    locs = g.random((nsets, k, 2))
    y = g.standard_normal((nsets, k)).cumsum(1) * 0.1
    nus = [0.5, 1.5, 2.5]
    slots = torch.tensor([0, 1, 2], dtype=torch.int32, device=DEV)
    feat, gam = api.variogram(torch.tensor(locs, device=DEV), torch.tensor(y, device=DEV), slots, 32, 0.5, 3,
                              nchunks=16)
    feat, gam = feat.cpu().numpy(), gam.cpu().numpy()
    for b in range(nsets):
        ref_g, ref_c = OLR.variogram(locs[b], y[b])
        np.testing.assert_allclose(gam[b], ref_g, rtol=1e-12, atol=0)
        np.testing.assert_allclose(feat[b], OLR.features(locs[b], y[b], nus[b]), rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
@pytest.mark.parametrize("bf16", [True, False])
def test_gemm_vs_oracle(ta, tb, bf16):
    from paper_2410_04477_amd import api
    M, N, K = 45, 37, 70   # ragged in every dimension
    g = W.rng(11)
    A = g.standard_normal((K, M) if ta else (M, K)).astype(np.float32)
    B = g.standard_normal((N, K) if tb else (K, N)).astype(np.float32)
    bias = g.standard_normal(N).astype(np.float32)
    C = torch.zeros((M, N), dtype=torch.float32, device=DEV)
    api.gemm(torch.tensor(A, device=DEV), torch.tensor(B, device=DEV), C, ta=ta, tb=tb,
             bias=torch.tensor(bias, device=DEV), bf16=bf16)
    rnd = OLR.bf16_round if bf16 else (lambda x: np.asarray(x, np.float64))
    Ao = rnd(A).T if ta else rnd(A)
    Bo = rnd(B).T if tb else rnd(B)
    ref = Ao @ Bo + bias
    np.testing.assert_allclose(C.cpu().numpy(), ref, rtol=1e-5, atol=1e-5 * np.abs(ref).max())


@pytest.mark.parametrize("bf16", [True, False])
def test_mlp_forward_backward_adam_vs_oracle(bf16):
    from paper_2410_04477_amd.warmstart import MLP
    from paper_2410_04477_amd import api
    B = 64
    g = W.rng(13)
    params = OLR.init_params(7)
    X = np.abs(g.standard_normal((B, 96))) * 0.5
    T = g.standard_normal((B, 3))
    net = MLP(0, DEV, bf16=bf16)
    net.set_params(params)
    p32 = [np.asarray(p, np.float32).astype(np.float64) for p in params]
    Xg = torch.tensor(X, dtype=torch.float32, device=DEV)
    Tg = torch.tensor(T, dtype=torch.float32, device=DEV)
    out, cache = net.forward(Xg)
    dout = torch.empty_like(out)
    part = api.mse(out, Tg, dout)
    grads = net.backward(cache, dout)
    rnd = OLR.bf16_round if bf16 else (lambda x: x)
    X32 = X.astype(np.float32).astype(np.float64)
    T32 = T.astype(np.float32).astype(np.float64)
    o_ref, c_ref = OLR.forward(p32, X32, rnd)
    loss_ref, g_ref = OLR.mse_backward(p32, c_ref, o_ref, T32, rnd)
    tol = 2e-3 if bf16 else 1e-5
    np.testing.assert_allclose(out.cpu().numpy(), o_ref, rtol=tol, atol=tol * np.abs(o_ref).max())
    assert float(part.sum()) == pytest.approx(loss_ref, rel=tol)
    for gg, gr in zip(grads, g_ref):
        gg = gg.cpu().numpy()
        assert np.linalg.norm(gg - gr) <= (5 * tol) * np.linalg.norm(gr) + 1e-12
    # one Adam step from zero state
    p_ref, _, _ = OLR.adam_step(p32, [np.asarray(x.cpu().numpy(), np.float64) for x in grads],
                                [np.zeros_like(p) for p in p32], [np.zeros_like(p) for p in p32], 1, lr=1e-3)
    for p, gr, m, v in zip(net.params, grads, net.m, net.v):
        api.adam(p, gr, m, v, 1, 1e-3)
    for p, pr in zip(net.params, p_ref):
        np.testing.assert_allclose(p.cpu().numpy(), pr, rtol=1e-5, atol=1e-6)


def _training_sets(ndesign, per_design, n, seed):
    from paper_2410_04477_amd import warmstart as WS
    feats, thetas = [], []
    for dsg in range(ndesign):
        locs = W.uniform_square(n, seed + dsg)
        order = W.point_permutation(n, seed + dsg)
        sub = W.subset_indices(n, 1024, seed + dsg)
        design = WS.make_design(locs, order, sub, sim_m=60)
        th = W.warm_thetas(per_design, seed * 1000 + dsg)
        z = torch.tensor(W.rng(seed + 77 * dsg).standard_normal((per_design, n)), device=DEV)
        ys = WS.simulate_sets(design, th, z)
        assert torch.isfinite(ys).all()
        feats.append(WS.features_for(design, ys, [t.nu for t in th]))
        thetas += th
    return torch.cat(feats, 0), thetas


def test_training_reduces_loss_and_warm_start_helps():
    from paper_2410_04477_amd import mle, warmstart as WS
    from paper_2410_04477_amd.model import BlockVecchia
    feats, thetas = _training_sets(4, 96, 3000, 900)
    net = WS.MLP(1, DEV)
    hist = net.fit(feats, thetas, epochs=120, batch=64, lr=2e-3, seed=1)
    assert hist[-1] < 0.5 * hist[0]
    # held-out data sets: warm start vs cold start MLE
    n = 6000
    evals_w, evals_c, gap = [], [], []
    th_test = W.warm_thetas(6, 4242)
    for i, th in enumerate(th_test):
        th = th.replace(nu=1.5)
        locs = W.uniform_square(n, 5000 + i)
        order = W.point_permutation(n, 5000 + i)
        design = WS.make_design(locs, order, W.subset_indices(n, 1024, 5000 + i), sim_m=60)
        z = torch.tensor(W.standard_normal(n, 6000 + i), device=DEV)[None]
        y_ord = WS.simulate_sets(design, [th], z)[0]
        feat = WS.features_for(design, y_ord[None], [th.nu])
        th_hat = tuple(net.predict(feat)[0])
        start = th_hat if WS.valid_theta(th_hat) else W.C4_THETA0
        y = y_ord.cpu().numpy()[np.argsort(order)]
        mod = BlockVecchia(locs, y, 600, 40, th.nu, W.kmeans_init(n, 600, i), W.block_permutation(600, i))
        rw = mle.fit(mod, start, "fp64", max_evals=120)
        rc = mle.fit(mod, W.C4_THETA0, "fp64", max_evals=120)
        evals_w.append(rw.evals)
        evals_c.append(rc.evals)
        gap.append((rw.loglik - rc.loglik) / abs(rc.loglik))
        # both fits end stationary by the FP64 adjoint (mle.fit restarts L-BFGS while they are not)
        assert rw.grad_eta <= 1e-6 and rc.grad_eta <= 1e-6, (rw, rc)
    print("warm evals", evals_w, "cold evals", evals_c, "rel loglik gap", gap)
    assert np.median(evals_w) <= np.median(evals_c)
    assert min(gap) >= -1e-6   # warm start ends at least as likely (to tolerance)
