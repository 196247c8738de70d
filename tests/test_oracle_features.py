"""Pins of the float64 placement-feature reference."""
import numpy as np

import oracle
from oracle import features
from paper_2305_08343_amd import scenes


def test_tri_thinness_closed_forms():
    s3 = np.sqrt(3.0)
    tris = np.array([
        [[0, 0, 0], [1, 0, 0], [0.5, s3 / 2, 0]],        # equilateral
        [[0, 0, 0], [1, 0, 0], [2, 0, 0]],               # degenerate (collinear)
        [[0, 0, 0], [0, 1, 0], [0, 0, 1]],               # right isosceles
        [[0, 0, 0], [4, 0, 0], [0, 0.1, 0]],             # thin
        [[1, 1, 1], [1, 1, 1], [1, 1, 1]],               # a point
    ])
    th = features.tri_thinness(tris)
    assert abs(th[0]) < 1e-12
    assert th[1] == 1.0
    assert np.isclose(th[2], 1 - 4 * s3 * 0.5 / 4.0)
    assert np.isclose(th[3], 1 - 4 * s3 * 0.2 / (16 + 0.01 + 16.01))
    assert th[4] == 1.0


def test_slot_features_invariants(small_scene, small_oracle):
    tris, _ = small_scene
    bvh = small_oracle["bvh"]
    f = features.slot_features(tris, bvh, small_oracle["masks6"], 6)
    assert f.shape == (2 * bvh.n_inner, 12)
    assert (f[:, 0:3] >= 0).all() and (f[:, 0:3] <= 1).all()
    # a child spanning its parent on an axis has ratio exactly 1 there
    box = bvh.cbox.reshape(-1, 2, 6).astype(np.float64)
    plo = np.minimum(box[:, 0, :3], box[:, 1, :3])
    phi = np.maximum(box[:, 0, 3:], box[:, 1, 3:])
    spans = (box[:, :, :3] == plo[:, None]) & (box[:, :, 3:] == phi[:, None]) & (phi > plo)[:, None]
    assert (f[:, 0:3].reshape(-1, 2, 3)[spans] == 1.0).all()
    assert (f[:, 3] <= 0).all() and (f[:, 4] > 0).all() and (f[:, 4] <= 1).all()
    leaf = (bvh.cref.reshape(-1) & 0x80000000) != 0
    assert (f[:, 11] == leaf).all()
    counts = np.where(leaf, ((bvh.cref.reshape(-1) >> 29) & 3) + 1,
                      bvh.range[np.where(leaf, 0, bvh.cref.reshape(-1) & 0x7FFFFFFF), 1])
    assert np.allclose(f[:, 5], np.log2(1 + counts) / 24)
    # strands are thin: mean thinness high
    assert f[:, 7].mean() > 0.5  # ribbon triangles 2e-3 x 9.4e-3: thinness ~0.64
    # box centres lie in the root box; the root's two children are on either side of its centre
    # on some axis, or share a centre there
    assert (f[:, 8:11] >= 0).all() and (f[:, 8:11] <= 1).all()
    mid = (box[0, :, :3] + box[0, :, 3:]) * 0.5
    assert np.allclose(f[0:2, 8:11], (mid - plo[0]) / (phi[0] - plo[0]))


def test_position_features_of_two_corner_triangles():
    """Three triangles in each of two opposite corners of the box [0, 10]^3: the root's children
    are the two corner leaves, with box centres (0.5, 0.5, 0) and (9.5, 9.5, 10), at positions
    (0.05, 0.05, 0) and (0.95, 0.95, 1) of the root box."""
    a = np.array([[[0, 0, 0], [1, 0, 0], [0, 1, 0]], [[1, 1, 0], [1, 0, 0], [0, 1, 0]],
                  [[0.5, 0.5, 0], [1, 0, 0], [0, 0, 0]]], np.float32)
    tris = np.concatenate([a, np.float32(10.0) - a]).astype(np.float32)
    bvh = oracle.bvh_build(tris)
    assert bvh.n_inner == 1
    f = features.slot_features(tris, bvh, np.zeros((2, 4), np.uint64), 6)
    pos = sorted(map(tuple, np.round(f[:, 8:11], 12)))
    assert pos == [(0.05, 0.05, 0.0), (0.95, 0.95, 1.0)]
    # a flat root box (every triangle in z = 3) gives position 0 on that axis
    flat = tris.copy()
    flat[..., 2] = 3.0
    fb = oracle.bvh_build(flat)
    ff = features.slot_features(flat, fb, np.zeros((2, 4), np.uint64), 6)
    assert (ff[:, 10] == 0.0).all()


def test_position_features_follow_mirror_and_affine_maps(small_scene):
    """Mirroring the scene on an axis maps that axis' position p to 1 - p (and the other features
    stay), scaling and translating it leaves the positions unchanged: pins the low-face origin,
    the axis order and the root extent used as the scale."""
    tris, _ = small_scene
    tris = np.asarray(tris, np.float32)
    bvh = oracle.bvh_build(tris)
    _, delta = oracle.default_bounds(tris)
    f = features.slot_features(tris, bvh, oracle.object_masks(tris, bvh, 6, delta), 6)
    # a power-of-two scale keeps every float32 box exact: the same tree, the same positions
    scaled = (tris * np.float32(4.0)).astype(np.float32)
    bs = oracle.bvh_build(scaled)
    fs = features.slot_features(scaled, bs, oracle.object_masks(scaled, bs, 6, delta * 4), 6)
    assert (bs.cref == bvh.cref).all()
    assert np.allclose(fs[:, 8:11], f[:, 8:11], rtol=0, atol=1e-12)
    # a translation rounds the coordinates: compare the sorted positions
    moved = (tris + np.array([8.0, -16.0, 2.0], np.float32)).astype(np.float32)
    bm = oracle.bvh_build(moved)
    fm = features.slot_features(moved, bm, oracle.object_masks(moved, bm, 6, delta), 6)
    assert fm.shape == f.shape
    for j in range(8, 11):
        assert np.allclose(np.sort(fm[:, j]), np.sort(f[:, j]), atol=1e-5)
    for ax in range(3):
        mir = tris.copy()
        mir[..., ax] = -mir[..., ax]
        bmir = oracle.bvh_build(mir)
        fmir = features.slot_features(mir, bmir, oracle.object_masks(mir, bmir, 6, delta), 6)
        # the mirrored tree pairs slots up to a swap of each node's children: compare sorted rows
        # of (extent ratios, area, depth, count, thinness, leaf) with the mirrored position
        key = lambda g: np.round(np.concatenate([g[:, [0, 1, 2, 3, 4, 5, 7, 11]], g[:, 8:11]], 1), 6)
        want = f.copy()
        want[:, 8 + ax] = 1.0 - want[:, 8 + ax]
        a = key(want)
        b = key(fmir)
        assert np.allclose(a[np.lexsort(a.T[::-1])], b[np.lexsort(b.T[::-1])], atol=1e-6)


def test_subtree_means_are_means(small_scene, small_oracle):
    tris, _ = small_scene
    bvh = small_oracle["bvh"]
    f = features.slot_features(tris, bvh, small_oracle["masks4"], 4)
    th = features.tri_thinness(np.asarray(tris)[bvh.perm])
    rng = np.random.default_rng(0)
    for s in rng.choice(2 * bvh.n_inner, 40, replace=False):
        ref = int(bvh.cref.reshape(-1)[s])
        if ref & 0x80000000:
            a, n = ref & 0x1FFFFFFF, ((ref >> 29) & 3) + 1
        else:
            a, n = (int(x) for x in bvh.range[ref])
        assert np.allclose(f[s, 7], th[a:a + n].mean())
