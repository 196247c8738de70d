"""Pins of the oracle's BVH builder (binned SAH, Sect. 4; cost of Eq. 1).

Invariants that any correct build must satisfy, checked independently of the
build code: partition of the triangles into leaves, exact boxes, leaf size,
contiguous DFS pre-order ranges, recorded depth, and optimality of every
chosen split among all binned candidates (recomputed here in float64 from
the centroids).
"""
import numpy as np
import pytest

import oracle
from paper_2305_08343_amd import scenes

LEAF = oracle.LEAF_BIT


def _ref_range(bvh, ref):
    if ref & LEAF:
        return ref & 0x1FFFFFFF, ((ref >> 29) & 3) + 1
    return int(bvh.range[ref, 0]), int(bvh.range[ref, 1])


def _tri_boxes(tris):
    return tris.min(axis=1), tris.max(axis=1)


def _check_tree(tris, bvh, leaf_max=4):
    n = tris.shape[0]
    lo, hi = _tri_boxes(tris)
    assert sorted(bvh.perm.tolist()) == list(range(n))
    seen = np.zeros(n, int)
    max_depth = 0
    stack = [(bvh.root, 1)]
    while stack:
        ref, lvl = stack.pop()
        if ref & LEAF:
            f, c = _ref_range(bvh, ref)
            assert 1 <= c <= leaf_max
            seen[f:f + c] += 1
            continue
        max_depth = max(max_depth, lvl)
        f, c = _ref_range(bvh, ref)
        assert c > leaf_max
        (lf, lc), (rf, rc) = (_ref_range(bvh, int(x)) for x in bvh.cref[ref])
        assert lf == f and rf == lf + lc and lc + rc == c
        # DFS pre-order: an inner left child is the next node
        if not bvh.cref[ref, 0] & LEAF:
            assert bvh.cref[ref, 0] == ref + 1
        for ch in range(2):
            cf, cc = _ref_range(bvh, int(bvh.cref[ref, ch]))
            ids = bvh.perm[cf:cf + cc]
            box = bvh.cbox[ref, 6 * ch:6 * ch + 6]
            assert (box[:3] == lo[ids].min(0)).all() and (box[3:] == hi[ids].max(0)).all()
            stack.append((int(bvh.cref[ref, ch]), lvl + 1))
    assert (seen == 1).all()
    assert max_depth == bvh.depth


def _sa(lo, hi):
    d = hi.astype(np.float64) - lo.astype(np.float64)
    return 2.0 * ((d[0] * d[1] + d[1] * d[2]) + d[2] * d[0])


def _check_split_optimal(tris, bvh, node, bins=32):
    lo, hi = _tri_boxes(tris)
    cen = (lo + hi) * np.float32(0.5)
    f, c = _ref_range(bvh, node)
    ids = bvh.perm[f:f + c]
    lf, lc = _ref_range(bvh, int(bvh.cref[node, 0]))
    left = set(bvh.perm[lf:lf + lc].tolist())
    chosen = _sa(lo[list(left)].min(0), hi[list(left)].max(0)) * len(left)
    right = [i for i in ids if i not in left]
    chosen += _sa(lo[right].min(0), hi[right].max(0)) * len(right)
    best = np.inf
    cb_lo, cb_hi = cen[ids].min(0), cen[ids].max(0)
    for a in range(3):
        if not cb_hi[a] > cb_lo[a]:
            continue
        scale = np.float32(bins) / np.float32(cb_hi[a] - cb_lo[a])
        fb = (cen[ids, a] - cb_lo[a]) * scale
        k = np.where(fb >= bins - 1, bins - 1, fb.astype(np.int64))
        for s in range(1, bins):
            L = ids[k < s]
            Rr = ids[k >= s]
            if len(L) == 0 or len(Rr) == 0:
                continue
            cost = _sa(lo[L].min(0), hi[L].max(0)) * len(L) + _sa(lo[Rr].min(0), hi[Rr].max(0)) * len(Rr)
            best = min(best, cost)
    if np.isfinite(best):
        assert chosen <= best * (1 + 1e-12), (node, chosen, best)


def test_small_scene_invariants(small_scene, small_oracle):
    tris, _ = small_scene
    _check_tree(tris, small_oracle["bvh"])


def test_small_scene_splits_are_sah_optimal(small_scene, small_oracle):
    tris, _ = small_scene
    bvh = small_oracle["bvh"]
    for node in range(0, bvh.n_inner, 7):
        _check_split_optimal(tris, bvh, node)


@pytest.mark.parametrize("seed", range(30))
def test_micro_scenes(seed):
    n = 1 + (seed * 7) % 64
    tris = scenes.micro_scene(seed, n)
    bvh = oracle.bvh_build(tris)
    if n <= 4:
        assert bvh.n_inner == 0 and bvh.root & LEAF
        assert _ref_range(bvh, bvh.root) == (0, n)
    else:
        _check_tree(tris, bvh)
        for node in range(bvh.n_inner):
            _check_split_optimal(tris, bvh, node)


def test_degenerate_centroids_fall_back_to_median():
    # eight copies of one triangle: every centroid equal, no binned split exists
    t = np.tile(np.array([[[0, 0, 0], [1, 0, 0], [0, 1, 0]]], np.float32), (8, 1, 1))
    bvh = oracle.bvh_build(t)
    assert bvh.n_inner == 1
    assert [_ref_range(bvh, int(x)) for x in bvh.cref[0]] == [(0, 4), (4, 4)]
    assert list(bvh.perm) == list(range(8))


def test_empty_and_depth_cap():
    bvh = oracle.bvh_build(np.zeros((0, 3, 3), np.float32))
    assert bvh.root == oracle.EMPTY_REF and bvh.n_inner == 0
    tris = scenes.scene_small(0)
    with pytest.raises(RuntimeError):
        oracle.bvh_build(tris, depth_cap=3)


def test_non_finite_rejected():
    t = np.zeros((5, 3, 3), np.float32)
    t[2, 1, 0] = np.nan
    with pytest.raises(RuntimeError):
        oracle.bvh_build(t)
