"""Pins of the oracle's quantised 4-wide child boxes.

The quantisation is a layout choice, not part of the paper: each 4-wide node
(the node of Sect. 3.2.4 with four child boxes) stores the minimum corner of
its children, one power-of-two step per axis and every child plane as an 8-bit
count of steps, rounded outward. What fixes it independently of the oracle's
own code:
  * a hand-worked node whose exponents, counts and decoded planes follow from
    the definition by arithmetic done on paper (below);
  * for every node of real collapses: each decoded box contains the exact
    child box (the property the traversal relies on), each decoded plane lies
    within one step (and the final rounding) of the exact one, the exponent is
    the smallest whose 255 steps cover the extent unless the float32 decode of
    255 steps at a smaller one falls short of the greatest child maximum, and
    the corner is an exact child plane;
  * hand-worked nodes whose child planes differ greatly in magnitude from the
    corner (where the double quotient alone would give a count whose decoded
    plane cuts into the child, or the covering step would fall short), with
    the counts worked out on paper;
  * Alg. 4 over the decoded boxes, plain and with masks built on the decoded
    boxes, returns the brute-force closest hit (closest hit and ties as in the
    binary traversal).
"""
import numpy as np
import pytest

import oracle
from paper_2305_08343_amd import scenes
from tests.test_oracle_trace import _aimed_rays

EMPTY = oracle.EMPTY_REF
LEAF = oracle.LEAF_BIT


def _hand_node():
    box4 = np.zeros((1, 4, 6), np.float32)
    box4[0, 0] = [0.1, -2.0, 5.0, 0.7, -1.0, 5.0]
    box4[0, 1] = [0.0, -1.5, 5.0, 1.0, 3.0, 5.0]
    ref4 = np.array([[LEAF | 0, LEAF | 1, EMPTY, EMPTY]], np.uint32)
    src4 = np.array([[0, 1, EMPTY, EMPTY]], np.uint32)
    return oracle.BVH4(box4, ref4, src4, 0, 1)


def test_hand_worked_node():
    # x: corner 0, extent 1: 255 * 2^-8 < 1 <= 255 * 2^-7, so the step is 2^-7 (bias 120).
    #    float32(0.1) / 2^-7 = 12.8000002 -> 12 -> 0.09375; float32(0.7) / 2^-7 = 89.5999985 -> 90
    #    -> 0.703125; child 1: 0 and 1 / 2^-7 = 128 exactly.
    # y: corner -2, extent 5: 255 * 2^-6 < 5 <= 255 * 2^-5, step 2^-5 (bias 122); offsets 0, 1, 0.5
    #    and 5 are whole steps (0, 32, 16, 160), so the planes decode exactly.
    # z: extent 0: the smallest exponent, -126 (bias 1), every count 0.
    qt = oracle.quantise4(_hand_node())
    assert qt.lo.tolist() == [[0.0, -2.0, 5.0]]
    assert qt.ebias.tolist() == [[120, 122, 1]]
    assert qt.q[0, 0].tolist() == [12, 0, 0, 90, 32, 0]
    assert qt.q[0, 1].tolist() == [0, 16, 0, 128, 160, 0]
    assert (qt.q[0, 2:] == 0).all() and (qt.dec[0, 2:] == 0).all()
    assert qt.dec[0, 0].tolist() == [0.09375, -2.0, 5.0, 0.703125, -1.0, 5.0]
    assert qt.dec[0, 1].tolist() == [0.0, -1.5, 5.0, 1.0, 3.0, 5.0]


def _dec32(corner, q, e):
    """The float32 decode of count q at step 2^e: exact product, one rounding of the sum."""
    return np.float32(np.float32(corner) + np.float32(np.float32(q) * np.float32(2.0 ** e)))


def test_mixed_magnitude_node_contains_children():
    # x: child 0 spans [-1, 1], so the corner is -1 and the step 2^-6 (255 * 2^-7 < 2 <= 255 * 2^-6).
    # Child 1 spans [-2^-60, 2^-60]. In double, -2^-60 - (-1) rounds to 1 and 2^-60 - (-1) to 1, so the
    # quotients give counts 64 and 64, decoding both planes to exactly 0.0 -- outside the child on the
    # minimum side. Checked with the decode itself, the minimum moves down to 63 (-0.015625) and the
    # maximum up to 65 (0.015625).
    box4 = np.zeros((1, 4, 6), np.float32)
    box4[0, 0] = [-1.0, -1.0, -1.0, 1.0, 1.0, 1.0]
    box4[0, 1] = [-2.0 ** -60, 0.0, 0.0, 2.0 ** -60, 0.5, 0.5]
    ref4 = np.array([[LEAF | 0, LEAF | 1, EMPTY, EMPTY]], np.uint32)
    b4 = oracle.BVH4(box4, ref4, np.array([[0, 1, EMPTY, EMPTY]], np.uint32), 0, 1)
    qt = oracle.quantise4(b4)
    assert qt.ebias[0, 0] == 127 - 6
    assert (qt.q[0, 1, 0], qt.q[0, 1, 3]) == (63, 65)
    assert (qt.dec[0, 1, 0], qt.dec[0, 1, 3]) == (-0.015625, 0.015625)
    _check_quant(b4, qt)


def test_exponent_raised_when_the_largest_count_falls_short():
    # x: corner -255 * 2^40 (child 0 spans [-255 * 2^40, -1]), greatest maximum 2^-40 (child 1 spans
    # [-1, 2^-40]). The extent 255 * 2^40 + 2^-40 rounds to 255 * 2^40 in double, so 2^40 would be the
    # covering step, but 255 steps from the corner decode to 0.0 < 2^-40. The step becomes 2^41: child 1's
    # maximum needs ceil(127.5) = 128 steps (decoded 2^40), its minimum floor(127.49...) = 127 steps
    # (decoded -2^40); child 0 keeps 0 and 128 (-1 + 255 * 2^40 = 127.49... * 2^41, rounded up).
    big = np.float32(255.0 * 2.0 ** 40)
    box4 = np.zeros((1, 4, 6), np.float32)
    box4[0, 0] = [-big, 0.0, 0.0, -1.0, 1.0, 1.0]
    box4[0, 1] = [-1.0, 0.0, 0.0, 2.0 ** -40, 1.0, 1.0]
    ref4 = np.array([[LEAF | 0, LEAF | 1, EMPTY, EMPTY]], np.uint32)
    b4 = oracle.BVH4(box4, ref4, np.array([[0, 1, EMPTY, EMPTY]], np.uint32), 0, 1)
    qt = oracle.quantise4(b4)
    assert qt.ebias[0, 0] == 127 + 41
    assert qt.q[0, 0, [0, 3]].tolist() == [0, 128]
    assert qt.q[0, 1, [0, 3]].tolist() == [127, 128]
    assert qt.dec[0, 1, 0] == -(2.0 ** 40) and qt.dec[0, 1, 3] == 2.0 ** 40
    _check_quant(b4, qt)


def _check_quant(b4, qt):
    used = b4.ref4 != EMPTY
    ex = b4.box4.astype(np.float64)
    dec = qt.dec.astype(np.float64)
    e = qt.ebias.astype(np.int64) - 127
    step = np.ldexp(1.0, e)                                    # [n4, 3]
    assert (qt.ebias >= 1).all()
    for m in range(b4.n4):
        u = used[m]
        lo = ex[m, u, :3].min(0)
        hi = ex[m, u, 3:].max(0)
        assert (qt.lo[m].astype(np.float64) == lo).all()       # the corner is an exact child plane
        ext = hi - lo
        assert (255.0 * step[m] >= ext).all()
        # the smallest covering exponent, raised only while the largest count decoded in
        # float32 falls short of the greatest child maximum
        for a in range(3):
            e0 = -126
            while e0 < 127 and 255.0 * 2.0 ** e0 < ext[a]:
                e0 += 1
            assert e[m, a] >= e0
            for k in range(e0, int(e[m, a])):
                assert _dec32(qt.lo[m, a], 255, k) < np.float32(hi[a])
        # containment, plane by plane
        assert (dec[m, u, :3] <= ex[m, u, :3]).all() and (dec[m, u, 3:] >= ex[m, u, 3:]).all()
        # within one step plus the float32 rounding of the decoded sum
        ulp = np.spacing(np.maximum(np.abs(ex[m, u]), np.abs(dec[m, u])).astype(np.float32)).astype(np.float64)
        st = np.concatenate([step[m], step[m]])[None, :]
        assert (np.abs(dec[m, u] - ex[m, u]) <= st + ulp).all()
        assert (qt.q[m, u, :3] <= qt.q[m, u, 3:]).all()
        assert (qt.q[m, ~u] == 0).all() and (qt.dec[m, ~u] == 0).all()


def test_quantised_boxes_small_scene(small_scene, small_oracle):
    b4 = oracle.bvh4_collapse(small_oracle["bvh"])
    qt = oracle.quantise4(b4)
    _check_quant(b4, qt)
    # the boxes really are coarsened somewhere (the test would be vacuous otherwise)
    used = b4.ref4 != EMPTY
    assert (qt.dec[used] != b4.box4[used]).mean() > 0.3


@pytest.mark.parametrize("seed", range(20))
def test_quantised_boxes_micro_scenes(seed):
    tris = scenes.micro_scene(seed, 1 + (seed * 11) % 64)
    b4 = oracle.bvh4_collapse(oracle.bvh_build(tris))
    _check_quant(b4, oracle.quantise4(b4))


def test_with_slot_boxes_replaces_only_used_slots(small_oracle):
    bvh = small_oracle["bvh"]
    b4 = oracle.bvh4_collapse(bvh)
    d4 = oracle.decoded_bvh4(b4, oracle.quantise4(b4))
    bq = oracle.with_slot_boxes(bvh, d4)
    slots = bq.cbox.reshape(-1, 6)
    orig = bvh.cbox.reshape(-1, 6)
    used = d4.ref4 != EMPTY
    s = d4.src4[used]
    assert (slots[s].view(np.uint32) == d4.box4[used].view(np.uint32)).all()
    rest = np.setdiff1d(np.arange(slots.shape[0]), s)
    assert (slots[rest].view(np.uint32) == orig[rest].view(np.uint32)).all()
    assert (bq.cref == bvh.cref).all() and (bq.range == bvh.range).all() and (bq.perm == bvh.perm).all()


def _same(h, prim, t):
    return (h.prim == prim).all() and (h.t.view(np.uint32) == t.view(np.uint32)).all()


@pytest.mark.parametrize("seed", range(24))
def test_decoded_traversal_micro_scenes(seed):
    n = 1 + (seed * 13) % 64
    tris = scenes.micro_scene(seed, n)
    rays = np.concatenate([_aimed_rays(tris, 300, seed), scenes.random_rays(100, seed)])
    bvh = oracle.bvh_build(tris)
    b4 = oracle.bvh4_collapse(bvh)
    d4 = oracle.decoded_bvh4(b4, oracle.quantise4(b4))
    ob, delta = oracle.default_bounds(tris)
    bp, bt = oracle.brute_closest(tris, rays)
    assert _same(oracle.trace4(tris, bvh, d4, rays), bp, bt)
    bq = oracle.with_slot_boxes(bvh, d4)
    for R in (4, 6):
        m = oracle.object_masks(tris, bq, R, delta)
        h = oracle.trace4(tris, bq, d4, rays, mode="raw", R=R, masks=m, origin_bound=ob)
        assert _same(h, bp, bt)


def test_decoded_traversal_small_scene(small_scene, small_oracle):
    tris, rays = small_scene
    rays = np.concatenate([rays, _aimed_rays(tris, 20000, 33)])
    bvh = small_oracle["bvh"]
    b4 = oracle.bvh4_collapse(bvh)
    d4 = oracle.decoded_bvh4(b4, oracle.quantise4(b4))
    bq = oracle.with_slot_boxes(bvh, d4)
    ob, delta = small_oracle["origin_bound"], small_oracle["delta"]
    exact = oracle.trace4(tris, bvh, b4, rays, origin_bound=ob)
    plain = oracle.trace4(tris, bq, d4, rays, origin_bound=ob)
    assert _same(plain, exact.prim, exact.t)
    assert plain.box_tests.sum() >= exact.box_tests.sum()     # coarser boxes are hit at least as often overall
    m6 = oracle.object_masks(tris, bq, 6, delta)
    raw = oracle.trace4(tris, bq, d4, rays, mode="raw", R=6, masks=m6, origin_bound=ob)
    assert _same(raw, exact.prim, exact.t)
    assert raw.mask_culls.sum() > 0 and (raw.box_tests <= plain.box_tests).all()


def _extreme_scenes():
    """A flat scene (every node has a zero extent in z: the smallest exponent, -126), and
    the same triangles scaled by 1e15 and 1e-8 (large and small exponents; far larger
    factors would overflow or underflow the float32 triangle test itself)."""
    base = scenes.isotropic_tris(7, 200, 0.2)
    flat = base.copy()
    flat[:, :, 2] = np.float32(0.5)
    return {"flat": flat, "huge": (base.astype(np.float64) * 1e15).astype(np.float32),
            "tiny": (base.astype(np.float64) * 1e-8).astype(np.float32)}


def extreme_case(name):
    """The scene and its rays: aimed and random rays of the unscaled scene with their origins
    scaled like the vertices (the same rays in scaled units)."""
    tris = _extreme_scenes()[name]
    base = tris if name == "flat" else scenes.isotropic_tris(7, 200, 0.2)
    rays = np.concatenate([_aimed_rays(base, 400, 5), scenes.random_rays(100, 5)])
    f = {"flat": 1.0, "huge": 1e15, "tiny": 1e-8}[name]
    rays[:, :3] = (rays[:, :3].astype(np.float64) * f).astype(np.float32)
    return tris, rays


@pytest.mark.parametrize("name", ["flat", "huge", "tiny"])
def test_quantised_boxes_extreme_scales(name):
    tris, rays = extreme_case(name)
    bvh = oracle.bvh_build(tris)
    b4 = oracle.bvh4_collapse(bvh)
    qt = oracle.quantise4(b4)
    _check_quant(b4, qt)
    e = qt.ebias.astype(int) - 127
    if name == "flat":
        assert (e[:, 2] == -126).all() and (qt.q[:, :, [2, 5]] == 0).all()
    elif name == "huge":
        assert e.max() > 30
    else:
        assert e.min() < -30
    d4 = oracle.decoded_bvh4(b4, qt)
    bp, bt = oracle.brute_closest(tris, rays)
    h = oracle.trace4(tris, oracle.with_slot_boxes(bvh, d4), d4, rays)
    exact = oracle.trace4(tris, bvh, b4, rays)
    assert (bp != oracle.NO_HIT).sum() > 200
    # decoded boxes keep the exact boxes' hits
    assert _same(h, exact.prim, exact.t)
    if name == "flat":
        # coplanar overlapping triangles: equal (or one-ulp apart) hit distances make the closest
        # triangle ambiguous, so only the hit distance is fixed (to the rounding of the triangle test)
        assert ((h.prim == oracle.NO_HIT) == (bp == oracle.NO_HIT)).all()
        assert np.allclose(h.t, bt, rtol=1e-6, atol=0)
    else:
        assert _same(h, bp, bt)


def mixed_magnitude_case(kind):
    """Eight triangles in two clusters of four, apart in y, so the BVH is one inner node over two
    leaves and the 4-wide root holds two children whose x ranges are those of the hand-worked
    nodes above: "low" [-1, 1] and [-2^-60, 2^-60] (counts from the double quotients would cut
    into the second child), "high" [-255 * 2^40, -1] and [-1, 2^-40] (the covering step would fall
    short of the second child's maximum). Rays aimed at the triangles plus random rays."""
    if kind == "low":
        xa, xb = (-1.0, 1.0), (-(2.0 ** -60), 2.0 ** -60)
    else:
        xa, xb = (-255.0 * 2.0 ** 40, -1.0), (-1.0, 2.0 ** -40)
    tris = []
    for k in range(4):
        z = 0.1 * k
        tris.append([[xa[0], 2.0, z], [xa[1], 2.5, z + 0.05], [0.5 * (xa[0] + xa[1]), 3.0, z + 0.1]])
        tris.append([[xb[0], 0.1 * k, z], [xb[1], 0.1 * k + 0.2, z + 0.05], [0.0, 0.1 * k + 0.4, z + 0.1]])
    tris = np.asarray(tris, np.float32)
    rays = np.concatenate([_aimed_rays(tris, 400, 9), scenes.random_rays(100, 9)])
    return tris, rays


@pytest.mark.parametrize("kind", ["low", "high"])
def test_mixed_magnitude_scene(kind):
    tris, rays = mixed_magnitude_case(kind)
    bvh = oracle.bvh_build(tris)
    b4 = oracle.bvh4_collapse(bvh)
    assert b4.n4 == 1 and (b4.ref4[0, :2] & LEAF).all() and (b4.ref4[0, 2:] == EMPTY).all()
    xs = sorted((float(b4.box4[0, c, 0]), float(b4.box4[0, c, 3])) for c in range(2))
    want = {"low": [(-1.0, 1.0), (-(2.0 ** -60), 2.0 ** -60)],
            "high": [(-255.0 * 2.0 ** 40, -1.0), (-1.0, 2.0 ** -40)]}[kind]
    assert xs == sorted(want)
    qt = oracle.quantise4(b4)
    _check_quant(b4, qt)
    d4 = oracle.decoded_bvh4(b4, qt)
    bp, bt = oracle.brute_closest(tris, rays)
    assert (bp != oracle.NO_HIT).sum() > 100
    h = oracle.trace4(tris, oracle.with_slot_boxes(bvh, d4), d4, rays)
    assert _same(h, bp, bt)
