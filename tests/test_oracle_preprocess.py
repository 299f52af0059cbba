"""Pins of the oracle's preprocessing (Section 2.1; Alg. 1 preprocessing):
Lloyd fixed point, valid block partition and order, and exact nearest
neighbours by brute force."""
import numpy as np
import pytest

import workloads as W
from oracle import preprocess as P


def test_kmeans_fixed_point_and_partition():
    n, bc = 1500, 60
    s = W.rng(1).random((n, 2))
    lab, cen = P.kmeans(s, [1.0, 1.0], W.kmeans_init(n, bc, 1), max_iter=200)
    # Lloyd fixed point: every point is nearest its own centroid ...
    d2 = ((s[:, None, :] - cen[None]) ** 2).sum(-1)
    assert np.all(d2[np.arange(n), lab] <= d2.min(1) + 1e-15)
    # ... and every centroid is the mean of its members
    for k in range(bc):
        np.testing.assert_allclose(cen[k], s[lab == k].mean(0), rtol=1e-12)
    perm, bp = P.order_blocks(lab, W.block_permutation(bc, 1))
    assert sorted(perm.tolist()) == list(range(n))
    assert bp[0] == 0 and bp[-1] == n and np.all(np.diff(bp) > 0)
    bperm = W.block_permutation(bc, 1)
    for i in range(bc):
        blk = perm[bp[i]:bp[i + 1]]
        assert np.all(lab[blk] == bperm[i])          # block i is cluster zeta(i)
        assert np.all(np.diff(blk) > 0)              # ascending original index


def test_kmeans_empty_cluster_reseed_hand_example():
    # duplicate initial centroids: every point ties between clusters 0 and 1
    # and goes to the lower index, so cluster 1 is empty after the first
    # assignment.  Update: c0 = mean(0, 1, 2, 10) = 3.25; cluster 1 is re-seeded
    # with the point farthest from its (updated) centroid, x = 10.  Reassign:
    # {0, 1, 2} -> 0, {10} -> 1; update c = (1, 10); no change -> stop.
    x = np.array([[0.0], [1.0], [2.0], [10.0]])
    lab, cen = P.kmeans(x, [1.0], np.array([0, 0]), max_iter=30)
    assert lab.tolist() == [0, 0, 0, 1]
    np.testing.assert_array_equal(cen[:, 0], [1.0, 10.0])


def test_kmeans_two_empty_clusters_take_farthest_points_in_order():
    # three copies of x = 0 as initial centroids: clusters 1 and 2 start empty.
    # After the update c0 = 33/5 = 6.6, squared distances to it are
    # (43.56, 31.36, 21.16, 11.56, 179.56): cluster 1 takes x = 20 (farthest),
    # cluster 2 the next, x = 0.  Then {0, 1, 2} -> 2, {10} -> 0, {20} -> 1,
    # c = (10, 20, 1), and the next assignment changes nothing.
    x = np.array([[0.0], [1.0], [2.0], [10.0], [20.0]])
    lab, cen = P.kmeans(x, [1.0], np.array([0, 0, 0]), max_iter=30)
    assert lab.tolist() == [2, 2, 2, 0, 1]
    np.testing.assert_array_equal(cen[:, 0], [10.0, 20.0, 1.0])
    # no cluster is lost and the result is a Lloyd fixed point
    d2 = (x - cen[:, 0][None, :]) ** 2
    assert np.all(d2[np.arange(5), lab] == d2.min(1))


def test_kmeans_inertia_nonincreasing():
    n, bc = 800, 40
    s = W.rng(2).random((n, 3)) * [1, 1, 0.2]
    w = [1.0, 1.0, 5.0]
    init = W.kmeans_init(n, bc, 2)
    prev = np.inf
    for it in (0, 1, 2, 4, 8):
        lab, cen = P.kmeans(s, w, init, max_iter=it)
        x = s * w
        inertia = ((x - cen[lab]) ** 2).sum() if it else ((x - x[init][lab]) ** 2).sum()
        assert inertia <= prev + 1e-12
        prev = inertia


def _brute(cen, x, pre, m):
    d = np.array([np.sum((cen - x[j]) ** 2) for j in range(pre)])
    o = sorted(range(pre), key=lambda j: (d[j], j))
    return o[:min(m, pre)]


def test_block_neighbors_bruteforce_and_prefix():
    n, bc, m = 700, 50, 25
    s = W.rng(3).random((n, 2))
    lab, _ = P.kmeans(s, [1, 1], W.kmeans_init(n, bc, 3))
    perm, bp = P.order_blocks(lab, W.block_permutation(bc, 3))
    lp = s[perm]
    nptr, nidx = P.block_neighbors(lp, bp, [1, 1], m)
    cen = P.block_centroids(lp, bp, [1, 1])
    for i in range(bc):
        row = nidx[nptr[i]:nptr[i + 1]]
        assert np.all(row < bp[i])
        assert row.tolist() == _brute(cen[i], lp, bp[i], m)
        # centroid is the block mean
        np.testing.assert_allclose(cen[i], lp[bp[i]:bp[i + 1]].mean(0), rtol=1e-13)
    # nested: the m-list is a prefix of the 2m-list
    nptr2, nidx2 = P.block_neighbors(lp, bp, [1, 1], 2 * m)
    for i in range(bc):
        a = nidx[nptr[i]:nptr[i + 1]]
        assert nidx2[nptr2[i]:nptr2[i] + len(a)].tolist() == a.tolist()


def test_tree_path_matches_brute_force():
    n, bc, m = 30_000, 1500, 40
    s = W.rng(4).random((n, 3)) * [1, 1, 0.2]
    w = np.array([1, 1, 5.0])
    lab, _ = P.kmeans(s, w, W.kmeans_init(n, bc, 4), max_iter=5)
    perm, bp = P.order_blocks(lab, W.block_permutation(bc, 4))
    lp = s[perm]
    cen = P.block_centroids(lp, bp, w)
    rows = P._block_neighbors_tree(lp * w, bp, cen, m)
    g = W.rng(5)
    for i in list(g.choice(bc, 60, replace=False)) + [bc - 1]:
        ref = P._knn_one(cen[i], (lp * w)[:bp[i]], min(m, bp[i]))
        assert rows[i].tolist() == ref.tolist()


def test_all_previous_neighbours():
    bp = np.array([0, 3, 5, 9])
    nptr, nidx = P.block_neighbors(np.zeros((9, 2)), bp, [1, 1], -1)
    assert nptr.tolist() == [0, 0, 3, 8]
    assert nidx.tolist() == [0, 1, 2, 0, 1, 2, 3, 4]
