"""Pins of the oracle's traversal (Alg. 4 with Alg. 1 and the AND test).

* brute force: the BVH closest hit equals a scan of all triangles with the
  same triangle test and tie rule (tiny scenes);
* the float32 triangle test agrees with a float64 linear solve wherever the
  hit is well conditioned;
* culling never changes the closest hit (Sect. 3.1.2: the AND only removes
  boxes the ray cannot hit inside), and per ray the counts order as
  none >= compressed >= raw;
* all-ones masks cull nothing and leave the counts of plain traversal;
* a recursive re-formulation of the traversal gives the same counts;
* the ray mask covers the exact ray segment inside the box.
"""
import numpy as np
import pytest

import oracle
from paper_2305_08343_amd import scenes

NO_HIT = oracle.NO_HIT
LEAF = oracle.LEAF_BIT


def _same_hits(a, b):
    return (a.prim == b.prim).all() and (a.t.view(np.uint32) == b.t.view(np.uint32)).all()


def _aimed_rays(tris, n, seed, spread=0.6):
    """Rays from random origins around the scene aimed at random triangle points."""
    rng = np.random.default_rng(seed)
    lo, hi = tris.reshape(-1, 3).min(0), tris.reshape(-1, 3).max(0)
    c, ext = 0.5 * (lo + hi), np.maximum(hi - lo, 1e-3)
    o = c + (rng.random((n, 3)) - 0.5) * ext * (1 + 2 * spread)
    t = rng.integers(0, tris.shape[0], n)
    w = rng.dirichlet([1, 1, 1], n)
    target = np.einsum("nk,nkj->nj", w, tris[t].astype(np.float64))
    d = target - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rays = np.zeros((n, 8), np.float32)
    rays[:, :3], rays[:, 4:7], rays[:, 7] = o, d, np.inf
    return rays


# ---------------------------------------------------------------- brute force
def test_small_scene_matches_brute_force(small_scene, small_oracle):
    tris, rays = small_scene
    h = oracle.trace(tris, small_oracle["bvh"], rays, mode="none")
    bp, bt = oracle.brute_closest(tris, rays)
    assert (h.prim == bp).all()
    assert (h.t.view(np.uint32) == bt.view(np.uint32)).all()


def test_small_scene_aimed_rays_match_brute_force(small_scene, small_oracle):
    tris, _ = small_scene
    rays = _aimed_rays(tris, 20000, 11)
    h = oracle.trace(tris, small_oracle["bvh"], rays, mode="none")
    bp, bt = oracle.brute_closest(tris, rays)
    assert (h.prim != NO_HIT).mean() > 0.5
    assert (h.prim == bp).all() and (h.t.view(np.uint32) == bt.view(np.uint32)).all()


@pytest.mark.parametrize("seed", range(100))
def test_micro_scenes_match_brute_force(seed):
    n = 1 + (seed * 13) % 64
    tris = scenes.micro_scene(seed, n)
    rays = np.concatenate([_aimed_rays(tris, 300, seed), scenes.random_rays(100, seed)])
    bvh = oracle.bvh_build(tris)
    ob, delta = oracle.default_bounds(tris)
    bp, bt = oracle.brute_closest(tris, rays)
    h = oracle.trace(tris, bvh, rays, mode="none")
    assert (h.prim == bp).all() and (h.t.view(np.uint32) == bt.view(np.uint32)).all()
    for R in (4, 6):
        m = oracle.object_masks(tris, bvh, R, delta)
        hc = oracle.trace(tris, bvh, rays, mode="raw", R=R, masks=m, origin_bound=ob)
        assert _same_hits(h, hc)
        assert (hc.box_tests <= h.box_tests).all() and (hc.tri_tests <= h.tri_tests).all()


# ------------------------------------------------------- triangle test in fp64
def test_triangle_test_agrees_with_fp64_solve(small_scene, small_oracle):
    tris, _ = small_scene
    rays = _aimed_rays(tris, 4000, 12)
    h = oracle.trace(tris, small_oracle["bvh"], rays, mode="none")
    hit = h.prim != NO_HIT
    T = tris[h.prim[hit]].astype(np.float64)
    r = rays[hit].astype(np.float64)
    # solve o + t d = v0 + u e1 + v e2
    A = np.stack([-r[:, 4:7], T[:, 1] - T[:, 0], T[:, 2] - T[:, 0]], axis=2)
    x = np.linalg.solve(A, (r[:, :3] - T[:, 0])[..., None])[..., 0]
    t, u, v = x[:, 0], x[:, 1], x[:, 2]
    cond = np.linalg.cond(A)
    good = cond < 1e4
    assert good.mean() > 0.9
    assert np.allclose(t[good], h.t[hit][good], rtol=1e-5, atol=0)
    tol = 1e-3
    assert (u[good] >= -tol).all() and (v[good] >= -tol).all() and (u[good] + v[good] <= 1 + tol).all()


def test_fp64_closest_hit_agrees_where_unambiguous(small_scene, small_oracle):
    tris, _ = small_scene
    rays = _aimed_rays(tris, 1500, 13)
    h = oracle.trace(tris, small_oracle["bvh"], rays, mode="none")
    T = tris.astype(np.float64)
    e1, e2 = T[:, 1] - T[:, 0], T[:, 2] - T[:, 0]
    agree = 0
    checked = 0
    for i in range(rays.shape[0]):
        o, d = rays[i, :3].astype(np.float64), rays[i, 4:7].astype(np.float64)
        P = np.cross(d, e2)
        det = np.einsum("ij,ij->i", e1, P)
        with np.errstate(divide="ignore", invalid="ignore"):
            S = o - T[:, 0]
            u = np.einsum("ij,ij->i", S, P) / det
            Q = np.cross(S, e1)
            v = (Q @ d) / det
            t = np.einsum("ij,ij->i", e2, Q) / det
        inside = (u > 1e-4) & (v > 1e-4) & (u + v < 1 - 1e-4) & (t > 0) & (np.abs(det) > 1e-9)
        edge = (u > -1e-4) & (v > -1e-4) & (u + v < 1 + 1e-4) & (t > 0)
        if not inside.any():
            continue
        j = np.flatnonzero(inside)[np.argmin(t[inside])]
        near_edge = edge & ~inside & (t < t[j] * (1 + 1e-4))
        if near_edge.any():
            continue
        if np.sum(inside & (t < t[j] * (1 + 1e-5))) > 1:
            continue
        checked += 1
        agree += int(h.prim[i] == j)
    assert checked > 1000
    assert agree == checked


# ---------------------------------------------------------- culling exactness
@pytest.mark.parametrize("R", [4, 6])
def test_culling_keeps_hits_and_reduces_counts(small_scene, small_oracle, R):
    tris, rays = small_scene
    rays = np.concatenate([rays, _aimed_rays(tris, 20000, 14)])
    bvh, ob = small_oracle["bvh"], small_oracle["origin_bound"]
    masks = small_oracle[f"masks{R}"]
    h0 = oracle.trace(tris, bvh, rays, mode="none")
    h1 = oracle.trace(tris, bvh, rays, mode="raw", R=R, masks=masks, origin_bound=ob)
    assert _same_hits(h0, h1)
    assert (h1.box_tests <= h0.box_tests).all() and (h1.tri_tests <= h0.tri_tests).all()
    assert (h1.mask_culls <= h1.mask_tests).all()
    # the counts drop by exactly the skipped subtrees: fewer tests overall
    assert h1.box_tests.sum() + h1.tri_tests.sum() < h0.box_tests.sum() + h0.tri_tests.sum()
    # with culling disabled, the mask layout traverses like plain
    h2 = oracle.trace(tris, bvh, rays, mode="raw", R=R, masks=masks, origin_bound=ob, cull=False)
    assert _same_hits(h0, h2) and (h2.box_tests == h0.box_tests).all()
    assert (h2.tri_tests == h0.tri_tests).all() and (h2.mask_tests == 0).all()


def test_compressed_sits_between_plain_and_raw(small_scene, small_oracle):
    tris, rays = small_scene
    rays = np.concatenate([rays, _aimed_rays(tris, 20000, 15)])
    bvh, ob = small_oracle["bvh"], small_oracle["origin_bound"]
    R = 6
    masks = small_oracle["masks6"]
    cb, idx = oracle.compress(masks, bvh.slot_boxes(), R, 256)
    h0 = oracle.trace(tris, bvh, rays, mode="none")
    hr = oracle.trace(tris, bvh, rays, mode="raw", R=R, masks=masks, origin_bound=ob)
    hl = oracle.trace(tris, bvh, rays, mode="lut", R=R, codebook=cb, cidx=idx, origin_bound=ob)
    assert _same_hits(h0, hl)
    for f in ("box_tests", "tri_tests"):
        assert (getattr(h0, f) >= getattr(hl, f)).all()
        assert (getattr(hl, f) >= getattr(hr, f)).all()


def test_all_ones_masks_cull_nothing(small_scene, small_oracle):
    """A full mask can never give a zero AND (the ray mask holds its entry
    cell), so it is not tested at all and the traversal equals plain."""
    tris, rays = small_scene
    bvh = small_oracle["bvh"]
    full = np.zeros_like(small_oracle["masks6"])
    for b in range(216):
        full[:, b >> 6] |= np.uint64(1) << np.uint64(b & 63)
    h0 = oracle.trace(tris, bvh, rays, mode="none")
    h1 = oracle.trace(tris, bvh, rays, mode="raw", R=6, masks=full)
    assert _same_hits(h0, h1)
    assert (h1.mask_culls == 0).all() and (h1.mask_tests == 0).all()
    assert (h1.box_tests == h0.box_tests).all() and (h1.tri_tests == h0.tri_tests).all()


def test_full_masks_are_not_tested(small_scene, small_oracle):
    """Replacing some masks by full masks removes exactly their tests and culls."""
    tris, rays = small_scene
    rays = np.concatenate([rays, _aimed_rays(tris, 10000, 21)])
    bvh, ob = small_oracle["bvh"], small_oracle["origin_bound"]
    m = small_oracle["masks4"].copy()
    h_raw = oracle.trace(tris, bvh, rays, mode="raw", R=4, masks=m, origin_bound=ob)
    sel = np.zeros(m.shape[0], bool)
    sel[::3] = True
    m2 = m.copy()
    m2[sel] = np.uint64(0xFFFFFFFFFFFFFFFF)
    h2 = oracle.trace(tris, bvh, rays, mode="raw", R=4, masks=m2, origin_bound=ob)
    placed = (~sel).astype(np.uint8)
    h3 = oracle.trace(tris, bvh, rays, mode="sparse", R=4, masks=m, placed=placed, origin_bound=ob)
    for f in ("prim", "box_tests", "tri_tests", "mask_tests", "mask_culls"):
        assert (getattr(h2, f) == getattr(h3, f)).all(), f
    assert (h2.box_tests >= h_raw.box_tests).all() and h2.mask_tests.sum() < h_raw.mask_tests.sum()


@pytest.mark.parametrize("R", [4, 6])
def test_sparse_placement_bounds(small_scene, small_oracle, R):
    """All slots placed = raw; none placed = plain; any placement keeps the hits
    and its counts lie between the two."""
    tris, rays = small_scene
    rays = np.concatenate([rays, _aimed_rays(tris, 10000, 22)])
    bvh, ob = small_oracle["bvh"], small_oracle["origin_bound"]
    m = small_oracle[f"masks{R}"]
    S = m.shape[0]
    h0 = oracle.trace(tris, bvh, rays, mode="none")
    hr = oracle.trace(tris, bvh, rays, mode="raw", R=R, masks=m, origin_bound=ob)
    ha = oracle.trace(tris, bvh, rays, mode="sparse", R=R, masks=m, placed=np.ones(S, np.uint8), origin_bound=ob)
    hn = oracle.trace(tris, bvh, rays, mode="sparse", R=R, masks=m, placed=np.zeros(S, np.uint8), origin_bound=ob)
    for f in ("prim", "box_tests", "tri_tests", "mask_tests", "mask_culls"):
        assert (getattr(ha, f) == getattr(hr, f)).all()
    assert (hn.box_tests == h0.box_tests).all() and (hn.mask_tests == 0).all()
    rng = np.random.default_rng(R)
    hp = oracle.trace(tris, bvh, rays, mode="sparse", R=R, masks=m,
                      placed=(rng.random(S) < 0.4).astype(np.uint8), origin_bound=ob)
    assert _same_hits(h0, hp)
    for f in ("box_tests", "tri_tests"):
        assert (getattr(h0, f) >= getattr(hp, f)).all() and (getattr(hp, f) >= getattr(hr, f)).all()


def test_origin_outside_bound_skips_masks(small_scene, small_oracle):
    tris, _ = small_scene
    rays = _aimed_rays(tris, 500, 16)
    far = rays.copy()
    far[:, :3] = far[:, :3] - 50.0 * far[:, 4:7]
    h = oracle.trace(tris, small_oracle["bvh"], far, mode="raw", R=6,
                     masks=small_oracle["masks6"], origin_bound=small_oracle["origin_bound"])
    assert (h.mask_tests == 0).all()


def test_invalid_rays_miss_with_zero_counts(small_scene, small_oracle):
    tris, rays = small_scene
    bad = np.repeat(rays[:1], 6, 0)
    bad[0, 0] = np.nan
    bad[1, 4:7] = 0.0
    bad[2, 3], bad[2, 7] = 2.0, 1.0      # tmin > tmax
    bad[3, 7] = np.nan
    bad[4, 5] = np.inf
    bad[5, 3] = -np.inf
    h = oracle.trace(tris, small_oracle["bvh"], bad, mode="none")
    assert (h.prim == NO_HIT).all() and np.isinf(h.t).all()
    assert (h.box_tests == 0).all() and (h.tri_tests == 0).all()


def test_empty_scene_and_single_leaf():
    rays = scenes.random_rays(64, 1)
    empty = np.zeros((0, 3, 3), np.float32)
    h = oracle.trace(empty, oracle.bvh_build(empty), rays)
    assert (h.prim == NO_HIT).all() and (h.tri_tests == 0).all()
    t = scenes.micro_scene(2, 3)
    bvh = oracle.bvh_build(t)
    h = oracle.trace(t, bvh, rays)
    assert (h.tri_tests == 3).all() and (h.box_tests == 0).all()


# ------------------------------------------- recursive re-formulation (counts)
def _recursive_trace(tris, bvh, ray, masks=None, lut=None, R=6, ob=np.inf):
    f32 = np.float32
    o = ray[:3].astype(f32)
    d = ray[4:7].astype(f32)
    tmin = f32(ray[3])
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        inv = f32(1) / d
    st = {"best": NO_HIT, "t": f32(ray[7]), "box": 0, "tri": 0}
    use_mask = masks is not None and max(abs(o)) <= ob
    bits = None if masks is None else oracle.mask_bits(masks, R)
    lbits = None if lut is None else oracle.mask_bits(lut, R)

    def cell(lo, hi, t):
        out = []
        with np.errstate(all="ignore"):
            for j in range(3):
                ext = f32(hi[j] - lo[j])
                s = f32(R) / ext if ext > 0 else f32(0)
                if np.isinf(s):
                    s = f32(0)
                p = f32(o[j] + f32(t * d[j]))
                u = f32(f32(p - lo[j]) * s)
                u = u if u > 0 else f32(0)
                u = u if u < R - 1 else f32(R - 1)
                out.append(int(u))
        return out

    def visit(ref, tn):
        if tn > st["t"]:
            return
        if ref & LEAF:
            first, cnt = ref & 0x1FFFFFFF, ((ref >> 29) & 3) + 1
            for j in range(first, first + cnt):
                st["tri"] += 1
                idx = int(bvh.perm[j])
                v = tris[idx].astype(f32)
                e1, e2 = f32(v[1] - v[0]), f32(v[2] - v[0])
                with np.errstate(all="ignore"):
                    P = np.array([d[1] * e2[2] - d[2] * e2[1], d[2] * e2[0] - d[0] * e2[2],
                                  d[0] * e2[1] - d[1] * e2[0]], f32)
                    det = f32(f32(e1[0] * P[0] + e1[1] * P[1]) + e1[2] * P[2])
                    if det == 0:
                        continue
                    idet = f32(1) / det
                    S = f32(o - v[0])
                    u = f32(f32(f32(S[0] * P[0] + S[1] * P[1]) + S[2] * P[2]) * idet)
                    if u < 0 or u > 1:
                        continue
                    Q = np.array([S[1] * e1[2] - S[2] * e1[1], S[2] * e1[0] - S[0] * e1[2],
                                  S[0] * e1[1] - S[1] * e1[0]], f32)
                    vv = f32(f32(f32(d[0] * Q[0] + d[1] * Q[1]) + d[2] * Q[2]) * idet)
                    if vv < 0 or f32(u + vv) > 1:
                        continue
                    t = f32(f32(f32(e2[0] * Q[0] + e2[1] * Q[1]) + e2[2] * Q[2]) * idet)
                if t < tmin or t > st["t"]:
                    continue
                if t < st["t"] or (t == st["t"] and idx < st["best"]):
                    st["t"], st["best"] = t, idx
            return
        res = []
        for c in range(2):
            lo = bvh.cbox[ref, 6 * c:6 * c + 3]
            hi = bvh.cbox[ref, 6 * c + 3:6 * c + 6]
            st["box"] += 1
            t0, t1 = tmin, st["t"]
            with np.errstate(all="ignore"):
                for j in range(3):
                    near, far = (hi[j], lo[j]) if np.signbit(inv[j]) else (lo[j], hi[j])
                    a = f32(f32(near - o[j]) * inv[j])
                    b = f32(f32(far - o[j]) * inv[j])
                    b = f32(b * f32(1.0000003576278687))
                    t0 = a if a > t0 else t0
                    t1 = b if b < t1 else t1
            ok = t0 <= t1
            if ok and use_mask:
                cb_, ce_ = cell(lo, hi, t0), cell(lo, hi, t1)
                key = 0
                for q in (*cb_, *ce_):
                    key = key * R + q
                if not (lbits[key] & bits[2 * ref + c]).any():
                    ok = False
            res.append((ok, t0))
        ch = bvh.cref[ref]
        if res[0][0] and res[1][0]:
            near = 1 if res[1][1] < res[0][1] else 0
            visit(int(ch[near]), res[near][1])
            visit(int(ch[1 - near]), res[1 - near][1])
        elif res[0][0]:
            visit(int(ch[0]), res[0][1])
        elif res[1][0]:
            visit(int(ch[1]), res[1][1])

    visit(bvh.root, tmin)
    return st


def test_recursive_formulation_counts(small_scene, small_oracle):
    tris, rays = small_scene
    sel = np.concatenate([_aimed_rays(tris, 150, 17), rays[::1024]])
    bvh = small_oracle["bvh"]
    for masks, lut, mode in ((None, None, "none"),
                             (small_oracle["masks6"], small_oracle["lut6"], "raw")):
        h = oracle.trace(tris, bvh, sel, mode=mode, R=6, masks=masks,
                         origin_bound=small_oracle["origin_bound"])
        for i in range(sel.shape[0]):
            st = _recursive_trace(tris, bvh, sel[i], masks, lut, 6, small_oracle["origin_bound"])
            assert st["best"] == h.prim[i]
            assert st["box"] == h.box_tests[i] and st["tri"] == h.tri_tests[i], i


# ----------------------------------------------------- ray-mask conservativeness
def test_ray_mask_covers_exact_segment():
    """float64 points of the exact in-box segment fall in delta-dilated voxels
    of the float32 ray mask (Alg. 1 plus the voxel dilation)."""
    rng = np.random.default_rng(18)
    for R in (4, 6):
        lut = oracle.raymask_lut(R)
        delta = 5 * 2.0 ** -16
        for _ in range(3000):
            lo = rng.uniform(-1, 1, 3).astype(np.float32)
            ext = np.exp(rng.uniform(np.log(1e-3), np.log(1.0), 3)).astype(np.float32)
            if rng.random() < 0.1:
                ext[rng.integers(0, 3)] = 0
            hi = (lo + ext).astype(np.float32)
            o = rng.uniform(-3, 3, 3).astype(np.float32)
            tgt = lo + rng.random(3) * ext
            d = (tgt - o)
            d = (d / np.linalg.norm(d)).astype(np.float32)
            o64, d64 = o.astype(np.float64), d.astype(np.float64)
            with np.errstate(divide="ignore", invalid="ignore"):
                a = (lo.astype(np.float64) - o64) / d64
                b = (hi.astype(np.float64) - o64) / d64
            a, b = np.nan_to_num(np.minimum(a, b), nan=-np.inf), np.nan_to_num(np.maximum(a, b), nan=np.inf)
            t0, t1 = max(0.0, a.max()), b.min()
            if not t0 <= t1:
                continue
            # float32 slab, as the traversal computes it
            inv = (np.float32(1) / d).astype(np.float32)
            with np.errstate(all="ignore"):
                fa = (lo - o) * inv
                fb = (hi - o) * inv
            ft0, ft1 = np.float32(0), np.float32(np.inf)
            for j in range(3):
                x, y = fa[j], fb[j]
                if x > y:
                    x, y = y, x
                y = np.float32(y * np.float32(1.0000003576278687))
                ft0 = x if x > ft0 else ft0
                ft1 = y if y < ft1 else ft1
            if not ft0 <= ft1:
                continue
            m = oracle.mask_bits(oracle.ray_mask(lo, hi, o, d, ft0, ft1, R, lut), R)
            s = np.linspace(t0, t1, 64)
            P = o64 + s[:, None] * d64
            w = ext.astype(np.float64) / R
            cen = lo.astype(np.float64)[None] + (np.arange(R)[:, None] + 0.5) * w[None]
            near = np.abs(P[:, None, :] - cen[None]) <= (0.5 * w + delta)[None, None, :]
            for p in range(P.shape[0]):
                xs, ys, zs = (np.flatnonzero(near[p, :, j]) for j in range(3))
                covered = any(m[x + R * y + R * R * z] for x in xs for y in ys for z in zs)
                assert covered


def test_negative_zero_direction_on_a_box_plane_keeps_the_hit():
    """A ray whose x direction is -0 and whose origin lies on the plane x = lo of
    a child box: with the near/far bounds chosen by the direction's sign, the
    box stays hit (0 * -inf is NaN on one bound only, and NaN never narrows the
    interval), so the triangle edge on that plane is found as by brute force."""
    tri = np.array([[[0.5, 0.4, 0.5], [0.5, 0.6, 0.5], [0.7, 0.5, 0.5]]], np.float32)
    far = np.array([[[5.0 + k, 5.0, 5.0], [5.2 + k, 5.0, 5.0], [5.0 + k, 5.2, 5.1]] for k in range(8)], np.float32)
    tris = np.concatenate([tri, far])
    ray = np.array([[0.5, 0.5, 0.0, 0.0, -0.0, 0.0, 1.0, np.inf]], np.float32)
    bp, bt = oracle.brute_closest(tris, ray)
    assert bp[0] == 0
    bvh = oracle.bvh_build(tris)
    assert not (bvh.root & LEAF)
    for h in (oracle.trace(tris, bvh, ray), oracle.trace4(tris, bvh, oracle.bvh4_collapse(bvh), ray)):
        assert h.prim[0] == 0 and h.t.view(np.uint32)[0] == bt.view(np.uint32)[0]
