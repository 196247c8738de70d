"""Masks on leaf slots only (the build option that keeps a testable mask only
where the child is a leaf): the oracle's helper gives every inner child's slot
the full mask and keeps the leaf slots' masks. Pinned by what that choice
implies, not by the helper's own arithmetic:
  * the full mask has exactly R^3 bits; leaf slots are unchanged;
  * a culled leaf child saves only triangle tests, so every ray's box tests
    equal those of the unculled traversal, exactly, on both BVH widths;
  * hits equal the unculled traversal's; triangle tests never exceed them;
  * in shadow mode no inner slot ever counts a false positive (its full
    mask is never tested), and every culled test sits on a leaf slot.
"""
import numpy as np
import pytest

import oracle


def _popcount(words):
    return sum(bin(int(w)).count("1") for w in words)


@pytest.mark.parametrize("R", [4, 6])
def test_helper_fills_inner_slots_and_keeps_leaf_slots(small_oracle, R):
    bvh = small_oracle["bvh"]
    masks = small_oracle[f"masks{R}"]
    out = oracle.leaf_slot_masks(masks, bvh, R)
    inner = (bvh.cref.reshape(-1) & oracle.LEAF_BIT) == 0
    W = oracle.words_for(R)
    m, o = masks.reshape(-1, W), out.reshape(-1, W)
    assert inner.any() and (~inner).any()
    assert (o[~inner] == m[~inner]).all()
    assert all(_popcount(row) == R ** 3 for row in o[inner][:200])
    assert (o[inner] == o[inner][0]).all()


@pytest.mark.parametrize("R", [4, 6])
def test_leaf_masks_cut_only_triangle_tests(small_scene, small_oracle, R):
    tris, rays = small_scene
    bvh = small_oracle["bvh"]
    ob = small_oracle["origin_bound"]
    lm = oracle.leaf_slot_masks(small_oracle[f"masks{R}"], bvh, R)
    b4 = oracle.bvh4_collapse(bvh)
    for width in (2, 4):
        if width == 2:
            none = oracle.trace(tris, bvh, rays, mode="none", origin_bound=ob)
            leaf = oracle.trace(tris, bvh, rays, mode="raw", R=R, masks=lm, origin_bound=ob)
        else:
            none = oracle.trace4(tris, bvh, b4, rays, mode="none", origin_bound=ob)
            leaf = oracle.trace4(tris, bvh, b4, rays, mode="raw", R=R, masks=lm, origin_bound=ob)
        assert (leaf.prim == none.prim).all() and (leaf.t.view(np.uint32) == none.t.view(np.uint32)).all()
        assert (leaf.box_tests == none.box_tests).all()
        assert (leaf.tri_tests <= none.tri_tests).all() and leaf.tri_tests.sum() < none.tri_tests.sum()
        assert leaf.mask_culls.sum() > 0


def test_shadow_false_positives_only_on_leaf_slots(small_scene, small_oracle):
    tris, rays = small_scene
    bvh = small_oracle["bvh"]
    lm = oracle.leaf_slot_masks(small_oracle["masks6"], bvh, 6)
    sh = oracle.trace(tris, bvh, rays, mode="raw", R=6, masks=lm, origin_bound=small_oracle["origin_bound"],
                      cull=False, shadow=True)
    inner = (bvh.cref.reshape(-1) & oracle.LEAF_BIT) == 0
    assert sh.slot_fp[inner].sum() == 0 and sh.slot_fp[~inner].sum() == sh.mask_culls.sum() > 0
