"""Pins of the oracle's block orderings: the Morton order of a regular grid
is the Z curve written out from its definition (bit interleaving of the
cell coordinates, checked against a hand-listed 4 x 4 sequence), the maxmin
order satisfies its defining property by brute force, and reordering keeps
every block intact; with the KL divergence (eq. (kl-gaussian-vecchia)) the
orderings are compared as in the paper's ordering study."""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle import loglik as OL, ordering as O, preprocess as P, simulate


def test_morton_order_of_a_grid_is_the_z_curve():
    # 4 x 4 cell centres; the Z curve visits (x, y) cells in this order
    g = np.array([(x, y) for y in range(4) for x in range(4)], dtype=float) + 0.5
    z = [(0, 0), (1, 0), (0, 1), (1, 1), (2, 0), (3, 0), (2, 1), (3, 1),
         (0, 2), (1, 2), (0, 3), (1, 3), (2, 2), (3, 2), (2, 3), (3, 3)]
    order = O.morton_order(g)
    got = [tuple(int(v) for v in g[i] - 0.5) for i in order]
    assert got == z


def test_morton_keys_3d_bits():
    cen = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0], [1.0, 1.0, 1.0]])
    k = O.morton_keys(cen)
    top = (1 << 21) - 1
    ref = [0]
    for axis in range(3):
        v = 0
        for b in range(21):
            v |= ((top >> b) & 1) << (3 * b + axis)
        ref.append(v)
    ref.append(ref[1] | ref[2] | ref[3])
    assert [int(v) for v in k] == ref


def test_maxmin_property_brute_force():
    g = W.rng(201)
    cen = g.random((60, 2))
    order = O.maxmin_order(cen)
    assert sorted(order.tolist()) == list(range(60))
    mean = cen.mean(0)
    d0 = ((cen - mean) ** 2).sum(1)
    assert order[0] == int(np.argmin(d0))
    for t in range(1, 60):
        placed = cen[order[:t]]
        mind = np.array([((placed - c) ** 2).sum(1).min() for c in cen])
        mind[order[:t]] = -1.0
        assert mind[order[t]] == pytest.approx(mind.max(), rel=1e-12)


@pytest.mark.parametrize("method", ["morton", "maxmin", "hilbert", "kdtree"])
def test_reorder_keeps_blocks(method):
    g = W.rng(202)
    s = g.random((300, 2))
    labels, _ = P.kmeans(s, [1.0, 1.0], W.kmeans_init(300, 30, 5))
    perm, bp = P.order_blocks(labels, W.block_permutation(30, 5))
    lp = s[perm]
    order, perm2, bp2 = O.reorder(lp, bp, [1.0, 1.0], method)
    for i, b in enumerate(order):
        assert np.array_equal(perm2[bp2[i]:bp2[i + 1]], np.arange(bp[b], bp[b + 1]))


def test_orderings_kl_properties_small():
    """The paper's ordering study in miniature (n = 600, 150 blocks): for
    every ordering KL >= 0 and KL falls as the nested neighbour sets grow
    (m = 5, 10, 20).  (Which ordering wins depends on the block count; at this
    size Morton has the smallest KL.)"""
    th = W.Theta(1.0, 0.1, 1e-4, 1.5)
    g = W.rng(203)
    s = g.random((600, 2))
    labels, _ = P.kmeans(s, [1.0, 1.0], W.kmeans_init(600, 150, 6))
    perm, bp = P.order_blocks(labels, W.block_permutation(150, 6))
    lp = s[perm]
    for method in ("random", "morton", "maxmin"):
        if method == "random":
            lpo, bpo = lp, bp
        else:
            _, p2, bpo = O.reorder(lp, bp, [1.0, 1.0], method)
            lpo = lp[p2]
        kls = []
        for m in (5, 10, 20):
            nptr, nidx = P.block_neighbors(lpo, bpo, [1.0, 1.0], m)
            kls.append(OL.kl_divergence(lpo, bpo, nptr, nidx, th))
        assert all(v >= -1e-9 for v in kls)
        assert kls[0] >= kls[1] - 1e-9 and kls[1] >= kls[2] - 1e-9


@pytest.mark.parametrize("d,k", [(2, 1), (2, 2), (2, 3), (2, 5), (3, 1), (3, 2), (3, 3)])
def test_hilbert_index_is_a_hilbert_curve(d, k):
    """The defining properties of a Hilbert curve on every 2^k grid: the
    indices of the 2^(kd) cells are a permutation of 0 .. 2^(kd) - 1, the
    curve starts at the origin, and cells with consecutive indices are
    neighbours (Manhattan distance 1).  With the full key width (B = 32 in
    2-D, 21 in 3-D) the first 2^(kd) indices fill the sub-grid at the origin."""
    pts = np.array(list(itertools.product(range(2 ** k), repeat=d)), dtype=np.uint64)
    for bits in (k, {2: 32, 3: 21}[d]):
        key = O.hilbert_index(pts, bits)
        assert np.array_equal(np.sort(key), np.arange(2 ** (k * d), dtype=np.uint64))
        c = pts[np.argsort(key)].astype(np.int64)
        assert not c[0].any()
        assert np.all(np.abs(np.diff(c, axis=0)).sum(1) == 1)


def test_hilbert_order_1d_and_locality():
    """1-D: the cell order.  2-D: blocks adjacent in the Hilbert order are on
    average closer than under a random order (locality of the curve)."""
    g = W.rng(204)
    x = g.random((50, 1))
    assert np.array_equal(O.hilbert_order(x), np.lexsort((np.arange(50), x[:, 0])))
    c = g.random((400, 2))
    steps = lambda o: np.linalg.norm(np.diff(c[o], axis=0), axis=1).mean()
    assert steps(O.hilbert_order(c)) < 0.25 * steps(g.permutation(400))


def test_kdtree_order_of_a_grid_and_split_property():
    """On a 4 x 4 grid (axis 0 split first, then axis 1, then axis 0 ...) the
    order is the nested quadrants: x < 2 before x >= 2, and within each half
    y < 2 before y >= 2, and so on down to single cells.  On random points
    every subtree holds a contiguous range split at the median."""
    pts = np.array([(x, y) for x in range(4) for y in range(4)], dtype=np.float64)
    o = O.kdtree_order(pts)
    c = pts[o]
    expect = [(0, 0), (0, 1), (1, 0), (1, 1), (0, 2), (0, 3), (1, 2), (1, 3),
              (2, 0), (2, 1), (3, 0), (3, 1), (2, 2), (2, 3), (3, 2), (3, 3)]
    assert [tuple(int(v) for v in r) for r in c] == expect
    g = W.rng(205)
    cen = g.random((37, 3))
    o = O.kdtree_order(cen)
    assert np.array_equal(np.sort(o), np.arange(37))

    def check(lo, hi, depth):
        if hi - lo <= 1:
            return
        axis, mid = depth % 3, lo + (hi - lo) // 2
        left, right = cen[o[lo:mid], axis], cen[o[mid:hi], axis]
        assert left.max() <= right.min()
        check(lo, mid, depth + 1)
        check(mid, hi, depth + 1)

    check(0, 37, 0)
