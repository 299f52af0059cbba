"""Learned warm start, FP64 reference: binned empirical semivariogram features
and a 96 -> 256 -> 256 -> 3 ReLU MLP (forward, backward, MSE, Adam).

Readings (the warm start is not in the paper; its shape is fixed by the
workload definition):
  * 32 equal-width distance bins on (0, h_max], h_max = 0.5; a pair (i, j),
    i < j, falls in bin floor(h / h_max * 32) (h == h_max goes to bin 31);
    pairs with h == 0 or h > h_max are skipped.  Pairs are all pairs of a
    seeded subset of points.
  * gamma_k = sum_{pairs in k} (y_i - y_j)^2 / (2 N_k); gamma_k = 0 when N_k = 0.
  * Features: gamma_k / s2, s2 = mean(y_sub^2) - mean(y_sub)^2 of the subset,
    placed in the slot of the data set's nu (one-hot over nu in {0.5,1.5,2.5}),
    i.e. x[slot*32 + k], zeros in the other two slots.
  * Targets: (log sigma2, log beta, log(nugget + 1e-4)), standardised.
"""
from __future__ import annotations

import numpy as np

NBINS = 32
HMAX = 0.5
NU_SLOTS = (0.5, 1.5, 2.5)
NUG_EPS = 1e-4


def variogram(locs_sub: np.ndarray, y_sub: np.ndarray, nbins: int = NBINS, hmax: float = HMAX):
    """Binned semivariogram (gamma, counts) over all pairs i < j of the subset."""
    k = locs_sub.shape[0]
    gsum = np.zeros(nbins)
    cnt = np.zeros(nbins, dtype=np.int64)
    for i in range(k - 1):
        dx = locs_sub[i + 1:] - locs_sub[i]
        h = np.sqrt(np.sum(dx * dx, axis=1))
        dy = y_sub[i + 1:] - y_sub[i]
        ok = (h > 0) & (h <= hmax)
        b = np.minimum((h[ok] / hmax * nbins).astype(np.int64), nbins - 1)
        np.add.at(gsum, b, dy[ok] ** 2)
        np.add.at(cnt, b, 1)
    gamma = np.where(cnt > 0, gsum / (2.0 * np.maximum(cnt, 1)), 0.0)
    return gamma, cnt


def features(locs_sub, y_sub, nu: float) -> np.ndarray:
    gamma, _ = variogram(locs_sub, y_sub)
    s2 = float(np.mean(y_sub * y_sub) - np.mean(y_sub) ** 2)
    x = np.zeros(3 * NBINS)
    slot = NU_SLOTS.index(nu)
    x[slot * NBINS:(slot + 1) * NBINS] = gamma / s2
    return x


def targets(sigma2, beta, nugget) -> np.ndarray:
    return np.array([np.log(sigma2), np.log(beta), np.log(nugget + NUG_EPS)])


def bf16_round(x):
    """Round to the nearest BF16 value (8-bit exponent, 8-bit significand,
    ties to even), returned as float64.  Used to give the oracle the same
    operand precision as a BF16 matrix product with FP32 accumulation."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _ident(x):
    return x


def init_params(seed: int, sizes=(96, 256, 256, 3)):
    """He-uniform initialisation (seeded) -- weights W_k are (out, in)."""
    g = np.random.Generator(np.random.PCG64(seed))
    ps = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        lim = np.sqrt(6.0 / a)
        ps.append(g.uniform(-lim, lim, (b, a)))
        ps.append(np.zeros(b))
    return ps


def forward(params, X, rnd=_ident):
    """X: batch x 96.  Returns (out, cache).  rnd rounds every matrix-product
    operand (identity = exact FP64)."""
    W1, b1, W2, b2, W3, b3 = params
    z1 = rnd(X) @ rnd(W1).T + b1
    a1 = np.maximum(z1, 0.0)
    z2 = rnd(a1) @ rnd(W2).T + b2
    a2 = np.maximum(z2, 0.0)
    out = rnd(a2) @ rnd(W3).T + b3
    return out, (X, z1, a1, z2, a2)


def mse_backward(params, cache, out, T, rnd=_ident):
    """Loss = mean over batch and outputs of (out - T)^2.  Returns (loss, grads).
    rnd rounds every matrix-product operand."""
    W1, b1, W2, b2, W3, b3 = params
    X, z1, a1, z2, a2 = cache
    diff = out - T
    loss = float(np.mean(diff * diff))
    dout = 2.0 * diff / diff.size
    gW3 = rnd(dout).T @ rnd(a2)
    gb3 = dout.sum(0)
    da2 = rnd(dout) @ rnd(W3)
    dz2 = da2 * (z2 > 0)
    gW2 = rnd(dz2).T @ rnd(a1)
    gb2 = dz2.sum(0)
    da1 = rnd(dz2) @ rnd(W2)
    dz1 = da1 * (z1 > 0)
    gW1 = rnd(dz1).T @ rnd(X)
    gb1 = dz1.sum(0)
    return loss, [gW1, gb1, gW2, gb2, gW3, gb3]


def adam_step(params, grads, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba), t = 1-based step count."""
    out_p, out_m, out_v = [], [], []
    for p, g, mm, vv in zip(params, grads, m, v):
        mm = b1 * mm + (1 - b1) * g
        vv = b2 * vv + (1 - b2) * g * g
        mh = mm / (1 - b1 ** t)
        vh = vv / (1 - b2 ** t)
        out_p.append(p - lr * mh / (np.sqrt(vh) + eps))
        out_m.append(mm)
        out_v.append(vv)
    return out_p, out_m, out_v
