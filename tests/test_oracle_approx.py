"""Pins of the oracle's approximate object masks (Sect. 3.2.1, Alg. 2).

* the filling-pattern table: every entry is the box of voxels between its two
  corner indices (count = product of the ranges; empty when a range is
  empty);
* Alg. 2 on hand-placed boxes: a child voxel fills exactly the parent voxels
  its extent (plus the 2 delta margin) projects to;
* conservativeness: at every level L the approximate mask contains the exact
  mask (so culling stays exact), on the strand scene and on micro scenes;
* L at least the subtree height gives the exact mask; leaf slots are exact at
  every L; hits under culling with approximate masks equal unculled hits,
  with counts between the exact-mask and the unculled ones.
"""
import numpy as np
import pytest

import oracle
from paper_2305_08343_amd import scenes


def _bits(m, R):
    return oracle.mask_bits(np.asarray(m, np.uint64)[None], R)[0]


def _voxels(m, R):
    b = _bits(m, R)
    return {(x, y, z) for z in range(R) for y in range(R) for x in range(R) if b[x + R * y + R * R * z]}


@pytest.mark.parametrize("R", [4, 6])
def test_fill_table_closed_form(R):
    t = oracle.fill_table(R)
    rng = np.random.default_rng(R)
    pc = np.unpackbits(t.view(np.uint8), axis=1).sum(1)
    for key in rng.integers(0, R ** 6, 500):
        k = int(key)
        z1 = k % R; k //= R
        y1 = k % R; k //= R
        x1 = k % R; k //= R
        z0 = k % R; k //= R
        y0 = k % R; k //= R
        x0 = k
        n = max(0, x1 - x0 + 1) * max(0, y1 - y0 + 1) * max(0, z1 - z0 + 1)
        assert pc[key] == n
        if n:
            vox = _voxels(t[key], R)
            assert min(v[0] for v in vox) == x0 and max(v[2] for v in vox) == z1
    full = ((((0 * R + 0) * R + 0) * R + R - 1) * R + R - 1) * R + R - 1
    assert pc[full] == R ** 3


def test_fill_one_hand_cases():
    R, delta = 4, 1e-4
    parent = [0, 0, 0, 1, 1, 1]
    cm = np.zeros(1, np.uint64)
    cm[0] = 1  # child voxel (0, 0, 0)
    child = [0.5, 0.5, 0.5, 1, 1, 1]  # child voxel (0,0,0) spans [0.5, 0.625]^3 -> parent 1..2 per axis
    out = oracle.fill_one(parent, cm, child, R, delta)
    assert _voxels(out, R) == {(x, y, z) for x in (1, 2) for y in (1, 2) for z in (1, 2)}
    cm[0] = np.uint64(1) << np.uint64(63)  # child voxel (3, 3, 3) spans [0.875, 1]^3 -> parent 3 only
    assert _voxels(oracle.fill_one(parent, cm, child, R, delta), R) == {(3, 3, 3)}
    # a zero-extent parent axis is filled whole, as the exact mask does
    flat = [0, 0, 0.5, 1, 1, 0.5]
    cm[0] = 1
    vox = _voxels(oracle.fill_one(flat, cm, [0.5, 0.5, 0.5, 1, 1, 0.5], R, delta), R)
    assert vox == {(x, y, z) for x in (1, 2) for y in (1, 2) for z in range(4)}


def _check_scene(tris, R, Ls):
    bvh = oracle.bvh_build(tris)
    ob, delta = oracle.default_bounds(tris)
    exact = oracle.object_masks(tris, bvh, R, delta)
    table = oracle.fill_table(R)
    leaf = (bvh.cref.reshape(-1) & oracle.LEAF_BIT) != 0
    out = {}
    for L in Ls:
        a = oracle.approx_masks(tris, bvh, R, delta, L, table)
        assert ((exact & ~a) == 0).all(), f"L={L}: not a superset of the exact mask"
        assert (a[leaf] == exact[leaf]).all()
        out[L] = a
    assert (oracle.approx_masks(tris, bvh, R, delta, 64, table) == exact).all()
    return bvh, ob, exact, out


@pytest.mark.parametrize("R", [4, 6])
def test_superset_and_exact_limit_small_scene(small_scene, R):
    tris, rays = small_scene
    bvh, ob, exact, approx = _check_scene(tris, R, (1, 2, 3, 4, 5))
    pc = {L: np.unpackbits(m.view(np.uint8), axis=1).sum() for L, m in approx.items()}
    assert pc[1] > pc[5] > np.unpackbits(exact.view(np.uint8), axis=1).sum()
    # culling with approximate masks: same hits, counts between exact masks and no masks
    none = oracle.trace(tris, bvh, rays, origin_bound=ob)
    ex = oracle.trace(tris, bvh, rays, mode="raw", R=R, masks=exact, origin_bound=ob)
    ap = oracle.trace(tris, bvh, rays, mode="raw", R=R, masks=approx[2], origin_bound=ob)
    assert (ap.prim == none.prim).all() and (ap.t.view(np.uint32) == none.t.view(np.uint32)).all()
    assert (ex.box_tests <= ap.box_tests).all() and (ap.box_tests <= none.box_tests).all()


@pytest.mark.parametrize("seed", range(30))
def test_superset_micro_scenes(seed):
    tris = scenes.micro_scene(seed, 1 + (seed * 11) % 64)
    _check_scene(tris, 6 if seed % 2 else 4, (1, 2, 3))
