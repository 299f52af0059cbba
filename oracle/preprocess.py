"""Preprocessing of Alg. 1: clustering g, block permutation zeta, and the
m nearest neighbours of each block centroid among earlier blocks
(Section 2.1 and Section 2.2, Alg. 1 preprocessing).

Readings where the paper is silent:
  * K-means is Lloyd's algorithm from given initial centroids (point indices
    passed in), in metric-scaled coordinates; it stops when no assignment
    changes or after max_iter iterations.  An empty cluster is re-seeded with
    the point farthest from its assigned centroid.  Any Lloyd fixed point is
    a correct answer: clusterings are compared by properties, not equality.
  * Within a block, points keep ascending original index.
  * Block centroid = arithmetic mean of the block's metric-scaled points,
    summed sequentially in block order, divided by the block size.
  * Neighbour distance: squared Euclidean distance in metric-scaled
    coordinates, evaluated as sum_k (c_k - s_k*w_k)^2 left to right without
    fused multiply-add; ties broken by lower (re-ordered) index.  m_i =
    min(m, number of earlier points); the first block has no neighbours.
    m = -1 means every earlier point (the exactness check).
"""
from __future__ import annotations

import numpy as np
from scipy.spatial import cKDTree


def _assign_brute(x: np.ndarray, c: np.ndarray) -> np.ndarray:
    out = np.empty(x.shape[0], dtype=np.int64)
    step = max(1, 4_000_000 // max(1, c.shape[0]))
    for a in range(0, x.shape[0], step):
        xs = x[a:a + step]
        d2 = ((xs[:, None, :] - c[None, :, :]) ** 2).sum(-1)
        out[a:a + step] = np.argmin(d2, axis=1)  # first minimum = lower index
    return out


def _assign(x: np.ndarray, c: np.ndarray) -> np.ndarray:
    if x.shape[0] * c.shape[0] <= 20_000_000:
        return _assign_brute(x, c)
    _, idx = cKDTree(c).query(x, k=1, workers=-1)
    return idx.astype(np.int64)


def kmeans(locs: np.ndarray, metric_scale, init_idx: np.ndarray, max_iter: int = 30):
    """Lloyd's K-means (clustering g, Section 2.1).  Returns (labels, centroids)
    in metric-scaled coordinates."""
    w = np.asarray(metric_scale, dtype=np.float64)
    x = locs * w
    c = x[init_idx].copy()
    bc = c.shape[0]
    labels = _assign(x, c)
    for _ in range(max_iter):
        counts = np.bincount(labels, minlength=bc)
        sums = np.zeros_like(c)
        for k in range(x.shape[1]):
            sums[:, k] = np.bincount(labels, weights=x[:, k], minlength=bc)
        nonempty = counts > 0
        c[nonempty] = sums[nonempty] / counts[nonempty, None]
        empty = np.flatnonzero(~nonempty)
        if empty.size:
            far = ((x - c[labels]) ** 2).sum(-1)
            order = np.argsort(-far, kind="stable")
            c[empty] = x[order[: empty.size]]
        new = _assign(x, c)
        changed = np.any(new != labels)
        labels = new
        if not changed and empty.size == 0:
            break
    return labels, c


def order_blocks(labels: np.ndarray, block_perm: np.ndarray):
    """Block permutation zeta (Section 2.1): position i holds cluster block_perm[i].
    Empty clusters are dropped.  Returns (perm new->old, block_ptr)."""
    n = labels.shape[0]
    bc = block_perm.shape[0]
    pos_of_label = np.empty(bc, dtype=np.int64)
    pos_of_label[block_perm] = np.arange(bc)
    pos = pos_of_label[labels]
    perm = np.lexsort((np.arange(n), pos)).astype(np.int64)  # by block position, then original index
    counts = np.bincount(pos, minlength=bc)
    counts = counts[counts > 0]
    block_ptr = np.zeros(counts.size + 1, dtype=np.int64)
    np.cumsum(counts, out=block_ptr[1:])
    return perm, block_ptr


def block_centroids(locs_perm: np.ndarray, block_ptr: np.ndarray, metric_scale) -> np.ndarray:
    """Mean of each block's metric-scaled points, summed sequentially in order."""
    w = np.asarray(metric_scale, dtype=np.float64)
    x = locs_perm * w
    bc = block_ptr.size - 1
    cen = np.empty((bc, x.shape[1]))
    for i in range(bc):
        a, b = block_ptr[i], block_ptr[i + 1]
        acc = np.zeros(x.shape[1])
        for j in range(a, b):
            acc = acc + x[j]
        cen[i] = acc / (b - a)
    return cen


def _sqdist(c: np.ndarray, x: np.ndarray) -> np.ndarray:
    t = c[None, :] - x
    out = t[:, 0] * t[:, 0]
    for k in range(1, x.shape[1]):
        out = out + t[:, k] * t[:, k]
    return out


def _knn_one(c, x_prefix, m):
    d2 = _sqdist(c, x_prefix)
    idx = np.arange(x_prefix.shape[0])
    o = np.lexsort((idx, d2))
    return o[:m]


def block_neighbors(locs_perm: np.ndarray, block_ptr: np.ndarray, metric_scale, m: int,
                    centroids: np.ndarray | None = None):
    """m nearest earlier points of each block centroid (Alg. 1, nearest neighbours).
    Returns (nbr_ptr, nbr_idx) as int64 CSR, each row sorted by (distance, index)."""
    w = np.asarray(metric_scale, dtype=np.float64)
    x = locs_perm * w
    bc = block_ptr.size - 1
    if centroids is None:
        centroids = block_centroids(locs_perm, block_ptr, metric_scale)
    rows = []
    if m < 0:
        rows = [np.arange(block_ptr[i], dtype=np.int64) for i in range(bc)]
    elif bc * block_ptr[-1] <= 50_000_000:
        for i in range(bc):
            pre = block_ptr[i]
            rows.append(_knn_one(centroids[i], x[:pre], min(m, pre)).astype(np.int64))
    else:
        rows = _block_neighbors_tree(x, block_ptr, centroids, m)
    counts = np.array([r.size for r in rows], dtype=np.int64)
    nbr_ptr = np.zeros(bc + 1, dtype=np.int64)
    np.cumsum(counts, out=nbr_ptr[1:])
    nbr_idx = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    return nbr_ptr, nbr_idx.astype(np.int64)


def _block_neighbors_tree(x, block_ptr, centroids, m):
    """Exact neighbours at scale: a KD-tree query of k' >> m nearest points of all
    blocks gives a candidate superset; the prefix condition and the exact
    (distance, index) order are then applied with the distance definition above.
    Blocks whose prefix candidates are not provably complete fall back to brute force."""
    bc = block_ptr.size - 1
    tree = cKDTree(x)
    kq = min(x.shape[0], 4 * m + 16)
    dist, idx = tree.query(centroids, k=kq, workers=-1)
    rows = []
    for i in range(bc):
        pre = int(block_ptr[i])
        mi = min(m, pre)
        if mi == 0:
            rows.append(np.zeros(0, np.int64))
            continue
        if pre <= 20_000:
            rows.append(_knn_one(centroids[i], x[:pre], mi).astype(np.int64))
            continue
        cand = idx[i][idx[i] < pre]
        ok = cand.size >= mi
        if ok:
            d2 = _sqdist(centroids[i], x[cand])
            o = np.lexsort((cand, d2))
            sel = cand[o[:mi]]
            # complete iff the m-th prefix distance is strictly inside the query ball
            ok = np.sqrt(d2[o[mi - 1]]) < dist[i][-1] * (1.0 - 1e-12)
        if ok:
            rows.append(sel.astype(np.int64))
        else:
            rows.append(_knn_one(centroids[i], x[:pre], mi).astype(np.int64))
    return rows


def point_neighbors(x_ordered: np.ndarray, m: int):
    """Classic Vecchia / simulator neighbours: for point i (in the given order),
    the min(m, i) nearest earlier points, sorted by (distance, index)."""
    n = x_ordered.shape[0]
    ptr = np.arange(n + 1, dtype=np.int64)
    return block_neighbors(x_ordered, ptr, np.ones(x_ordered.shape[1]), m, centroids=x_ordered)


def preprocess(locs, metric_scale, init_idx, block_perm, m, max_iter=30):
    """Full preprocessing of Alg. 1: clustering, block permutation, neighbours.
    Returns dict with perm, block_ptr, nbr_ptr, nbr_idx, locs_perm."""
    labels, _ = kmeans(locs, metric_scale, init_idx, max_iter)
    perm, block_ptr = order_blocks(labels, block_perm)
    locs_perm = locs[perm]
    nbr_ptr, nbr_idx = block_neighbors(locs_perm, block_ptr, metric_scale, m)
    return dict(perm=perm, block_ptr=block_ptr, nbr_ptr=nbr_ptr, nbr_idx=nbr_idx, locs_perm=locs_perm)
