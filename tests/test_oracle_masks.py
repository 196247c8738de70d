"""Pins of the oracle's object masks (Sect. 3.1.1, 3.2.1 with L = infinity).

A node's mask must be conservative (every voxel that any descendant triangle
touches is set) and tight up to the dilation delta (no voxel is set unless a
triangle comes within delta of it). Both are checked in float64 by sampling
the triangles, independently of the separating-axis code. A closed-form case
fixes the bit order x + R*y + R^2*z.
"""
import numpy as np
import pytest

import oracle
from paper_2305_08343_amd import scenes

LEAF = oracle.LEAF_BIT


def _slot_tris(bvh, slot):
    ref = int(bvh.cref[slot // 2, slot % 2])
    if ref & LEAF:
        f, c = ref & 0x1FFFFFFF, ((ref >> 29) & 3) + 1
    else:
        f, c = bvh.range[ref]
    return bvh.perm[f:f + c]


def _bary_samples(k):
    a, b = np.meshgrid(np.arange(k + 1), np.arange(k + 1), indexing="ij")
    keep = a + b <= k
    a, b = a[keep] / k, b[keep] / k
    return np.stack([1 - a - b, a, b], 1)  # [m, 3]


def test_closed_form_axis_aligned_triangle():
    # right triangle x+y <= 0.7, x,y >= 0.1 in the plane z = 0.3, box [0,1]^3, R = 4:
    # layer z = 1 only; cells (i,j) whose square meets the triangle
    tri = np.array([[0.1, 0.1, 0.3], [0.6, 0.1, 0.3], [0.1, 0.6, 0.3]], np.float32)
    m = oracle.voxelize_tri(tri, [0, 0, 0], [1, 1, 1], 4, 1e-6)
    bits = oracle.mask_bits(m, 4)
    expect = {(0, 0), (1, 0), (2, 0), (0, 1), (1, 1), (0, 2)}
    got = {(b % 4, (b // 4) % 4) for b in np.flatnonzero(bits)}
    assert got == expect
    assert {b // 16 for b in np.flatnonzero(bits)} == {1}


def test_closed_form_flat_box_sets_whole_column():
    # a triangle whose own box is flat in z: every z layer shares the same voxels
    tri = np.array([[0.1, 0.1, 0.3], [0.6, 0.1, 0.3], [0.1, 0.6, 0.3]], np.float32)
    m = oracle.voxelize_tri(tri, tri.min(0), tri.max(0), 4, 1e-6)
    bits = oracle.mask_bits(m, 4).reshape(4, 4, 4)  # [z, y, x]
    for z in range(4):
        assert (bits[z] == bits[0]).all()
    # in its own 4x4 grid over [0.1,0.6]^2 the hypotenuse passes the corners i+j = 4
    ij = {(x, y) for y in range(4) for x in range(4) if bits[0, y, x]}
    assert ij == {(x, y) for x in range(4) for y in range(4) if x + y <= 4}


def _check_conservative(tris, bvh, masks, R, delta, slots, k=24):
    bits = oracle.mask_bits(masks, R)
    bary = _bary_samples(k)
    for s in slots:
        ids = _slot_tris(bvh, s)
        box = bvh.cbox[s // 2, 6 * (s % 2):6 * (s % 2) + 6].astype(np.float64)
        lo, hi = box[:3], box[3:]
        w = (hi - lo) / R
        P = np.einsum("mk,tkj->tmj", bary, tris[ids].astype(np.float64)).reshape(-1, 3)
        # voxels whose (delta/2)-dilated box contains a sample must be set
        need = np.zeros(R ** 3, bool)
        centres = lo[None, :] + (np.arange(R)[:, None] + 0.5) * w[None, :]  # [R, 3]
        near = np.abs(P[:, None, :] - centres[None]) <= (0.5 * w + 0.5 * delta)[None, None, :]
        for x in range(R):
            for y in range(R):
                for z in range(R):
                    if (near[:, x, 0] & near[:, y, 1] & near[:, z, 2]).any():
                        need[x + R * y + R * R * z] = True
        assert not (need & ~bits[s]).any(), s


def _dist_point_box(P, lo, hi):
    d = np.maximum(np.maximum(lo - P, 0.0), P - hi)
    return np.abs(d).max(-1)


def _check_tight(tris, bvh, masks, R, delta, slots, k=48):
    bits = oracle.mask_bits(masks, R)
    bary = _bary_samples(k)
    for s in slots:
        ids = _slot_tris(bvh, s)
        box = bvh.cbox[s // 2, 6 * (s % 2):6 * (s % 2) + 6].astype(np.float64)
        lo, hi = box[:3], box[3:]
        w = (hi - lo) / R
        t64 = tris[ids].astype(np.float64)
        P = np.einsum("mk,tkj->tmj", bary, t64).reshape(-1, 3)
        edge = np.abs(t64[:, [1, 2, 0]] - t64).max()
        tol = delta + edge / k + 1e-6
        for b in np.flatnonzero(bits[s]):
            v = np.array([b % R, (b // R) % R, b // (R * R)])
            vlo, vhi = lo + v * w, lo + (v + 1) * w
            assert _dist_point_box(P, vlo, vhi).min() <= tol, (s, b)


def test_small_scene_conservative(small_scene, small_oracle):
    tris, _ = small_scene
    bvh = small_oracle["bvh"]
    rng = np.random.default_rng(0)
    # all leaf-level slots plus a random sample of upper slots
    small = [s for s in range(2 * bvh.n_inner) if len(_slot_tris(bvh, s)) <= 8]
    big = [s for s in range(2 * bvh.n_inner) if len(_slot_tris(bvh, s)) > 8]
    slots = small[::3] + list(rng.choice(big, 20, replace=False))
    for R, key in ((4, "masks4"), (6, "masks6")):
        _check_conservative(tris, bvh, small_oracle[key], R, small_oracle["delta"], slots)


def test_small_scene_tight(small_scene, small_oracle):
    tris, _ = small_scene
    bvh = small_oracle["bvh"]
    small = [s for s in range(2 * bvh.n_inner) if len(_slot_tris(bvh, s)) <= 16]
    for R, key in ((4, "masks4"), (6, "masks6")):
        _check_tight(tris, bvh, small_oracle[key], R, small_oracle["delta"], small[::5])


def test_masks_nest_with_hierarchy(small_oracle):
    """A child's occupied voxels lie inside the parent's: every set child
    voxel overlaps some set voxel of the parent's grid (both are conservative
    covers of the same triangles)."""
    bvh = small_oracle["bvh"]
    R = 4
    bits = oracle.mask_bits(small_oracle["masks4"], R)
    for node in range(1, bvh.n_inner, 5):
        # find the parent slot of this inner node
        where = np.argwhere(bvh.cref == node)
        if len(where) == 0:
            continue
        ps = 2 * where[0, 0] + where[0, 1]
        pbox = bvh.cbox[ps // 2, 6 * (ps % 2):6 * (ps % 2) + 6].astype(np.float64)
        pw = (pbox[3:] - pbox[:3]) / R
        for c in range(2):
            cs = 2 * node + c
            cbox = bvh.cbox[node, 6 * c:6 * c + 6].astype(np.float64)
            cw = (cbox[3:] - cbox[:3]) / R
            for b in np.flatnonzero(bits[cs]):
                v = np.array([b % R, (b // R) % R, b // (R * R)])
                vlo, vhi = cbox[:3] + v * cw, cbox[:3] + (v + 1) * cw
                ok = False
                for pb in np.flatnonzero(bits[ps]):
                    u = np.array([pb % R, (pb // R) % R, pb // (R * R)])
                    ulo = pbox[:3] + u * pw - 2 * small_oracle["delta"]
                    uhi = pbox[:3] + (u + 1) * pw + 2 * small_oracle["delta"]
                    if (vlo <= uhi).all() and (vhi >= ulo).all():
                        ok = True
                        break
                assert ok


@pytest.mark.parametrize("seed", range(12))
def test_micro_scene_masks(seed):
    tris = scenes.micro_scene(seed, 5 + seed * 4)
    bvh = oracle.bvh_build(tris)
    ob, delta = oracle.default_bounds(tris)
    for R in (4, 6):
        m = oracle.object_masks(tris, bvh, R, delta)
        slots = list(range(2 * bvh.n_inner))
        _check_conservative(tris, bvh, m, R, delta, slots, k=12)
        _check_tight(tris, bvh, m, R, delta, slots, k=24)


@pytest.mark.parametrize("R", [4, 6])
def test_slot_masks_equal_rows_of_all_slot_masks(small_scene, small_oracle, R):
    """The per-slot builder (used to check sampled slots of large scenes) gives exactly the
    rows of the all-slot builder, for slot lists that mix child 0 and child 1, leaf and inner
    children, the root's slots, repeated and unsorted slots, and the empty list."""
    tris, _ = small_scene
    bvh = small_oracle["bvh"]
    full = small_oracle[f"masks{R}"]
    S = 2 * bvh.n_inner
    leaf = (bvh.cref.reshape(-1) & np.uint32(oracle.LEAF_BIT)) != 0
    rng = np.random.default_rng(R)
    picks = [
        np.arange(4),                                                 # root's and its children's slots
        rng.integers(0, S, 500),                                       # random, repeats, any order
        rng.choice(np.flatnonzero(leaf), 200),                         # leaf children only
        rng.choice(np.flatnonzero(~leaf), 200),                        # inner children only
        np.array([S - 1, 0, S - 2, 1]),                                # last slots first
    ]
    for slots in picks:
        slots = np.asarray(slots, np.uint32)
        assert (slots % 2 == 0).any() and (slots % 2 == 1).any()
        got = oracle.slot_masks(tris, bvh, slots, R, small_oracle["delta"])
        assert got.shape == (slots.size, oracle.words_for(R))
        assert (got == full[slots]).all()
    assert oracle.slot_masks(tris, bvh, np.zeros(0, np.uint32), R, small_oracle["delta"]).shape[0] == 0


@pytest.mark.parametrize("seed", range(6))
def test_slot_masks_micro_scenes(seed):
    tris = scenes.micro_scene(seed, 5 + (seed * 17) % 60)
    bvh = oracle.bvh_build(tris)
    if bvh.n_inner == 0:
        pytest.skip("a single leaf has no child slots")
    _, delta = oracle.default_bounds(tris)
    full = oracle.object_masks(tris, bvh, 6, delta)
    slots = np.arange(2 * bvh.n_inner, dtype=np.uint32)[::-1].copy()
    assert (oracle.slot_masks(tris, bvh, slots, 6, delta) == full[slots]).all()
