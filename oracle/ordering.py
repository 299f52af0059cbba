"""Block orderings (Section 2.1: Morton, Hilbert, KD-tree and maxmin reorderings of the
blocks),
numpy FP64.  The KL divergence used to compare them (eq.
(kl-gaussian-vecchia)) is loglik.kl_divergence.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings where the paper is silent:
  * Blocks are ordered by their centroids (the mean of the block's metric-
    scaled points, as for the neighbour search).
  * Morton: each centroid coordinate is mapped to an integer cell on a grid of
    2^B cells per axis over the centroids' bounding box (B = 32 in 2-D, 21 in
    3-D, 63 bits in 1-D), cell = min(floor((c - lo) / (hi - lo) * 2^B), 2^B - 1);
    the key interleaves the bits, axis 0 in the lowest position; blocks are
    sorted by key, ties by block index.
  * Hilbert: the same cells as Morton, mapped to their distance along a
    Hilbert curve of order B by Skilling's transform (J. Skilling,
    "Programming the Hilbert curve", AIP Conf. Proc. 707, 2004): from the top
    bit down, undo the curve's rotations and reflections, Gray-encode, then
    read the index bits level by level, axis 0 most significant within a
    level.  In 1-D the curve is the cell order itself.  Sorted like Morton.
  * KD-tree: a k-d tree over the centroids built by median splits with the
    axis cycling with depth (axis = depth mod d, as in Bentley's tree); a
    node's blocks are sorted by (coordinate on that axis, block index), the
    first floor(k/2) go to the left child, and the order is that of the
    single-block leaves from left to right.
  * Maxmin: the first block is the one whose centroid is nearest the mean of
    the centroids (summed in block order); each next block maximises the minimum squared distance to
    the blocks already placed; ties by lowest block index.  Squared distances
    are summed over the axes left to right without fused multiply-add.
"""
from __future__ import annotations

import numpy as np

from .preprocess import _sqdist, block_centroids


def morton_keys(cen: np.ndarray) -> np.ndarray:
    """64-bit interleaved cell indices of the points (rows of cen)."""
    n, d = cen.shape
    bits = {1: 63, 2: 32, 3: 21}[d]
    lo, hi = cen.min(0), cen.max(0)
    ext = np.where(hi > lo, hi - lo, 1.0)
    scale = float(1 << bits)
    cells = np.minimum(np.floor((cen - lo) / ext * scale), scale - 1).astype(np.uint64)
    keys = np.zeros(n, dtype=np.uint64)
    for b in range(bits):
        for k in range(d):
            keys |= ((cells[:, k] >> np.uint64(b)) & np.uint64(1)) << np.uint64(b * d + k)
    return keys


def _cells(cen: np.ndarray):
    n, d = cen.shape
    bits = {1: 63, 2: 32, 3: 21}[d]
    lo, hi = cen.min(0), cen.max(0)
    ext = np.where(hi > lo, hi - lo, 1.0)
    scale = float(1 << bits)
    return np.minimum(np.floor((cen - lo) / ext * scale), scale - 1).astype(np.uint64), bits


def hilbert_index(cells: np.ndarray, bits: int) -> np.ndarray:
    """Distance along the order-`bits` Hilbert curve of integer cells (rows of
    an n x d uint64 array, each coordinate below 2^bits)."""
    n, d = cells.shape
    if d == 1:
        return cells[:, 0].astype(np.uint64)
    X = [cells[:, k].astype(np.uint64).copy() for k in range(d)]
    q = 1 << (bits - 1)
    while q > 1:
        Q, P = np.uint64(q), np.uint64(q - 1)
        for i in range(d):
            hit = (X[i] & Q) != 0
            X[0] = np.where(hit, X[0] ^ P, X[0])                 # reflect
            t = np.where(hit, np.uint64(0), (X[0] ^ X[i]) & P)    # or swap axes 0 and i
            X[0] = X[0] ^ t
            X[i] = X[i] ^ t
        q >>= 1
    for i in range(1, d):                                         # Gray encode
        X[i] = X[i] ^ X[i - 1]
    t = np.zeros(n, dtype=np.uint64)
    q = 1 << (bits - 1)
    while q > 1:
        t = np.where((X[d - 1] & np.uint64(q)) != 0, t ^ np.uint64(q - 1), t)
        q >>= 1
    for i in range(d):
        X[i] = X[i] ^ t
    key = np.zeros(n, dtype=np.uint64)
    for b in range(bits - 1, -1, -1):
        for i in range(d):
            key = (key << np.uint64(1)) | ((X[i] >> np.uint64(b)) & np.uint64(1))
    return key


def hilbert_order(cen: np.ndarray) -> np.ndarray:
    cells, bits = _cells(cen)
    keys = hilbert_index(cells, bits)
    return np.lexsort((np.arange(cen.shape[0]), keys))


def kdtree_order(cen: np.ndarray) -> np.ndarray:
    d = cen.shape[1]

    def visit(idx: np.ndarray, depth: int) -> list:
        if idx.size <= 1:
            return list(idx)
        axis = depth % d
        srt = idx[np.lexsort((idx, cen[idx, axis]))]
        mid = idx.size // 2
        return visit(srt[:mid], depth + 1) + visit(srt[mid:], depth + 1)

    return np.array(visit(np.arange(cen.shape[0]), 0), dtype=np.int64)


def morton_order(cen: np.ndarray) -> np.ndarray:
    keys = morton_keys(cen)
    return np.lexsort((np.arange(cen.shape[0]), keys))


def maxmin_order(cen: np.ndarray) -> np.ndarray:
    n = cen.shape[0]
    acc = np.zeros(cen.shape[1])
    for i in range(n):            # summed in order, like the centroids themselves
        acc = acc + cen[i]
    mean = acc / n
    first = int(np.lexsort((np.arange(n), _sqdist(mean, cen)))[0])
    order = [first]
    mind = _sqdist(cen[first], cen)
    placed = np.zeros(n, dtype=bool)
    placed[first] = True
    for _ in range(n - 1):
        cand = np.where(placed, -1.0, mind)
        nxt = int(np.argmax(cand))          # first index of the maximum
        order.append(nxt)
        placed[nxt] = True
        mind = np.minimum(mind, _sqdist(cen[nxt], cen))
    return np.array(order, dtype=np.int64)


def reorder(locs_perm: np.ndarray, block_ptr: np.ndarray, metric_scale, method: str):
    """New block order of blocks already in some order: returns (order, point
    permutation into locs_perm, new block_ptr)."""
    cen = block_centroids(locs_perm, block_ptr, metric_scale)
    order = {"morton": morton_order, "maxmin": maxmin_order, "hilbert": hilbert_order,
             "kdtree": kdtree_order}[method](cen)
    sizes = np.diff(block_ptr)[order]
    bp = np.zeros(order.size + 1, dtype=np.int64)
    np.cumsum(sizes, out=bp[1:])
    perm = np.concatenate([np.arange(block_ptr[b], block_ptr[b + 1]) for b in order]).astype(np.int64)
    return order, perm, bp

