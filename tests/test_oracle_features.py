"""Pins of the float64 placement-feature reference."""
import numpy as np

import oracle
from oracle import features
from paper_2305_08343_amd import scenes


def test_tri_shape_closed_forms():
    s3 = np.sqrt(3.0)
    tris = np.array([
        [[0, 0, 0], [1, 0, 0], [0.5, s3 / 2, 0]],        # equilateral
        [[0, 0, 0], [1, 0, 0], [2, 0, 0]],               # degenerate (collinear)
        [[0, 0, 0], [0, 1, 0], [0, 0, 1]],               # right isosceles, longest edge (0,-1,1)
        [[0, 0, 0], [4, 0, 0], [0, 0.1, 0]],             # thin, longest edge ~ x
    ])
    sh = features.tri_shape(tris)
    assert abs(sh[0, 0]) < 1e-12
    assert sh[1, 0] == 1.0
    assert np.isclose(sh[2, 0], 1 - 4 * s3 * 0.5 / 4.0)
    assert np.allclose(sh[2, 1:], [0, 1 / np.sqrt(2), 1 / np.sqrt(2)])
    L = np.hypot(4, 0.1)
    assert np.allclose(sh[3, 1:], [4 / L, 0.1 / L, 0])
    assert sh[3, 0] > 0.9


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
    # strands are thin: mean thinness high; direction cosines are unit-norm per triangle
    assert f[:, 7].mean() > 0.5  # ribbon triangles 2e-3 x 9.4e-3: thinness ~0.64
    sh = features.tri_shape(tris)
    assert np.allclose((sh[:, 1:] ** 2).sum(1), 1.0)


def test_subtree_means_are_means(small_scene, small_oracle):
    tris, _ = small_scene
    bvh = small_oracle["bvh"]
    f = features.slot_features(tris, bvh, small_oracle["masks4"], 4)
    sh = features.tri_shape(np.asarray(tris)[bvh.perm])
    rng = np.random.default_rng(0)
    for s in rng.choice(2 * bvh.n_inner, 40, replace=False):
        ref = int(bvh.cref.reshape(-1)[s])
        if ref & 0x80000000:
            a, n = ref & 0x1FFFFFFF, ((ref >> 29) & 3) + 1
        else:
            a, n = (int(x) for x in bvh.range[ref])
        assert np.allclose(f[s, 7:11], sh[a:a + n].mean(0))
