"""Pins of the oracle's 4-wide BVH (the node of Sect. 3.2.4 with four child
boxes and four child masks) and of Alg. 4 on it.

Collapse:
  * every used child box is the binary box of the slot it came from, bit for
    bit; used slots come first; a node keeps fewer than four children only
    when none of them can be expanded (all leaves);
  * every binary leaf is reached exactly once, nodes are in DFS pre-order;
  * the expansion rule as an inequality: every binary inner node absorbed
    into a 4-wide node has a surface area at least that of every binary
    inner child the node kept unexpanded (child boxes nest, so a greedy
    largest-area expansion implies it).
Traversal:
  * the closest hit equals the brute-force scan (small strand scene, aimed
    rays, micro scenes) and the binary traversal's hit;
  * culling never changes the hit; per ray, counts with masks never exceed
    the counts without them, and culls never exceed tests;
  * a recursive reformulation reproduces every per-ray count.
"""
import numpy as np
import pytest

import oracle
from paper_2305_08343_amd import scenes
from tests.test_oracle_trace import _aimed_rays

NO_HIT = oracle.NO_HIT
LEAF = oracle.LEAF_BIT
EMPTY = oracle.EMPTY_REF


def _slot_area(bvh, s):
    b = bvh.cbox[s >> 1, 6 * (s & 1):6 * (s & 1) + 6].astype(np.float64)
    d = b[3:] - b[:3]
    return 2.0 * ((d[0] * d[1] + d[1] * d[2]) + d[2] * d[0])


def _check_collapse(bvh, b4):
    if bvh.n_inner == 0:
        assert b4.n4 == 0 and b4.root == bvh.root
        return
    assert 1 <= b4.n4 <= bvh.n_inner
    # binary leaves reached from the 4-wide root, in order, exactly once; pre-order numbering
    seen_nodes, leaves4 = [], []
    bin_root = {b4.root: bvh.root}   # 4-wide node -> binary inner node it grew from

    def walk(m):
        seen_nodes.append(m)
        used = [c for c in range(4) if b4.ref4[m, c] != EMPTY]
        k = len(used)
        assert used == list(range(k)) and 2 <= k <= 4
        for c in range(k, 4):
            assert b4.src4[m, c] == EMPTY
        for c in range(k):
            s = int(b4.src4[m, c])
            assert (b4.box4[m, c].view(np.uint32) ==
                    bvh.cbox[s >> 1, 6 * (s & 1):6 * (s & 1) + 6].view(np.uint32)).all()
            r = int(bvh.cref[s >> 1, s & 1])
            if r & LEAF:
                assert b4.ref4[m, c] == r
                leaves4.append(r)
            else:
                if k < 4:
                    raise AssertionError(f"node {m} kept {k} children with an inner one")
                child = int(b4.ref4[m, c])
                bin_root[child] = r
                walk(child)
        # expansion rule: absorbed binary inner nodes vs unexpanded inner children
        kept = {int(b4.src4[m, c]) for c in range(k)}
        absorbed, stack = [], [bin_root[m]]
        while stack:
            node = stack.pop()
            for c in range(2):
                s = 2 * node + c
                if s in kept:
                    continue
                r = int(bvh.cref[node, c])
                assert not (r & LEAF), "a leaf must end up as a kept child"
                absorbed.append(s)
                stack.append(r)
        open_inner = [s for s in kept if not (int(bvh.cref[s >> 1, s & 1]) & LEAF)]
        if absorbed and open_inner:
            assert min(_slot_area(bvh, s) for s in absorbed) >= max(_slot_area(bvh, s) for s in open_inner)
        assert len(absorbed) == k - 2

    walk(b4.root)
    assert seen_nodes == list(range(b4.n4))
    bin_leaves = sorted(int(r) for r in bvh.cref.ravel() if r & LEAF)
    assert sorted(leaves4) == bin_leaves


def test_collapse_small_scene(small_oracle):
    b4 = oracle.bvh4_collapse(small_oracle["bvh"])
    _check_collapse(small_oracle["bvh"], b4)
    # each binary inner node seeds one 4-wide node or is absorbed into exactly one:
    # a node with k children holds k - 1 of them
    k = (b4.ref4 != EMPTY).sum(1)
    assert int((k - 1).sum()) == small_oracle["bvh"].n_inner
    assert b4.n4 < small_oracle["bvh"].n_inner and (k == 4).mean() > 0.3


@pytest.mark.parametrize("seed", range(40))
def test_collapse_micro_scenes(seed):
    tris = scenes.micro_scene(seed, 1 + (seed * 7) % 64)
    bvh = oracle.bvh_build(tris)
    _check_collapse(bvh, oracle.bvh4_collapse(bvh))


def test_collapse_of_leaf_and_empty_roots():
    for n in (0, 3):
        tris = scenes.micro_scene(5, n) if n else np.zeros((0, 3, 3), np.float32)
        bvh = oracle.bvh_build(tris)
        b4 = oracle.bvh4_collapse(bvh)
        assert b4.n4 == 0 and b4.root == bvh.root


def _same_hits(a, b):
    return (a.prim == b.prim).all() and (a.t.view(np.uint32) == b.t.view(np.uint32)).all()


def test_bvh4_matches_brute_force_and_binary(small_scene, small_oracle):
    tris, rays = small_scene
    rays = np.concatenate([rays, _aimed_rays(tris, 20000, 31)])
    bvh = small_oracle["bvh"]
    b4 = oracle.bvh4_collapse(bvh)
    h4 = oracle.trace4(tris, bvh, b4, rays)
    bp, bt = oracle.brute_closest(tris, rays)
    assert (h4.prim == bp).all() and (h4.t.view(np.uint32) == bt.view(np.uint32)).all()
    assert _same_hits(h4, oracle.trace(tris, bvh, rays))
    assert (h4.prim != NO_HIT).mean() > 0.2


@pytest.mark.parametrize("seed", range(60))
def test_bvh4_micro_scenes(seed):
    n = 1 + (seed * 13) % 64
    tris = scenes.micro_scene(seed, n)
    rays = np.concatenate([_aimed_rays(tris, 300, seed), scenes.random_rays(100, seed)])
    bvh = oracle.bvh_build(tris)
    b4 = oracle.bvh4_collapse(bvh)
    ob, delta = oracle.default_bounds(tris)
    bp, bt = oracle.brute_closest(tris, rays)
    h = oracle.trace4(tris, bvh, b4, rays)
    assert (h.prim == bp).all() and (h.t.view(np.uint32) == bt.view(np.uint32)).all()
    for R in (4, 6):
        m = oracle.object_masks(tris, bvh, R, delta)
        hc = oracle.trace4(tris, bvh, b4, rays, mode="raw", R=R, masks=m, origin_bound=ob)
        assert _same_hits(h, hc)


@pytest.mark.parametrize("R", [4, 6])
def test_bvh4_culling_keeps_hits_and_reduces_counts(small_scene, small_oracle, R):
    tris, rays = small_scene
    rays = np.concatenate([rays, _aimed_rays(tris, 20000, 32)])
    bvh = small_oracle["bvh"]
    b4 = oracle.bvh4_collapse(bvh)
    kw = dict(origin_bound=small_oracle["origin_bound"])
    plain = oracle.trace4(tris, bvh, b4, rays, **kw)
    raw = oracle.trace4(tris, bvh, b4, rays, mode="raw", R=R, masks=small_oracle[f"masks{R}"], **kw)
    cb, idx = oracle.compress(small_oracle[f"masks{R}"], bvh.slot_boxes(), R, 256)
    lut = oracle.trace4(tris, bvh, b4, rays, mode="lut", R=R, codebook=cb, cidx=idx, **kw)
    for h in (raw, lut):
        assert _same_hits(plain, h)
        assert (h.mask_culls <= h.mask_tests).all()
    assert (plain.box_tests >= lut.box_tests).all() and (lut.box_tests >= raw.box_tests).all()
    assert (plain.tri_tests >= lut.tri_tests).all() and (lut.tri_tests >= raw.tri_tests).all()
    assert raw.mask_culls.sum() > 0 and (raw.box_tests + raw.tri_tests).sum() < (plain.box_tests + plain.tri_tests).sum()


def _recursive_trace4(tris, bvh, b4, ray, masks=None, lut=None, R=6, ob=np.inf, test_max=None, cidx=None):
    """Alg. 4 on the 4-wide BVH as recursion: children sorted by (t0, index); a mask with more
    than test_max set bits (default R^3 - 1: only a full mask) is not tested. With cidx (the
    codebook index of each slot, masks then being the slots' codebook entries), st["refs"]
    counts the tests that read each codebook index."""
    f32 = np.float32
    o, d, tmin = ray[:3].astype(f32), ray[4:7].astype(f32), f32(ray[3])
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        inv = f32(1) / d
    st = {"best": NO_HIT, "t": f32(ray[7]), "box": 0, "tri": 0, "mt": 0, "mc": 0, "deep": 0, "refs": {}}
    use_mask = masks is not None and max(abs(o)) <= ob
    bits = None if masks is None else oracle.mask_bits(masks, R)
    lbits = None if lut is None else oracle.mask_bits(lut, R)
    limit = R ** 3 - 1 if test_max is None else test_max

    def cell(lo, hi, t):
        out = []
        with np.errstate(all="ignore"):
            for j in range(3):
                ext = f32(hi[j] - lo[j])
                s = f32(R) / ext if ext > 0 else f32(0)
                if np.isinf(s):
                    s = f32(0)
                u = f32(f32(f32(o[j] + f32(t * d[j])) - lo[j]) * s)
                u = u if u > 0 else f32(0)
                u = u if u < R - 1 else f32(R - 1)
                out.append(int(u))
        return out

    def leaf(ref):
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

    def visit(ref, tn, pending):
        # pending: children that an iterative traversal would hold on its stack beneath this
        # node -- the not yet visited siblings of every node on the recursion path
        if tn > st["t"]:
            return
        st["deep"] = max(st["deep"], pending)
        if ref & LEAF:
            leaf(ref)
            return
        alive = []
        for c in range(4):
            if b4.ref4[ref, c] == EMPTY:
                continue
            lo, hi = b4.box4[ref, c, :3], b4.box4[ref, c, 3:]
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
            if not t0 <= t1:
                continue
            s = int(b4.src4[ref, c])
            if use_mask and bits[s].sum() <= limit:
                st["mt"] += 1
                if cidx is not None:
                    st["refs"][int(cidx[s])] = st["refs"].get(int(cidx[s]), 0) + 1
                key = 0
                for q in (*cell(lo, hi, t0), *cell(lo, hi, t1)):
                    key = key * R + q
                if not (lbits[key] & bits[s]).any():
                    st["mc"] += 1
                    continue
            alive.append((t0, c))
        for i, (t0, c) in enumerate(sorted(alive)):
            visit(int(b4.ref4[ref, c]), t0, pending + len(alive) - 1 - i)

    visit(b4.root, tmin, 0)
    return st


def test_recursive_formulation_counts_bvh4(small_scene, small_oracle):
    tris, rays = small_scene
    sel = np.concatenate([_aimed_rays(tris, 150, 37), rays[::1024]])
    bvh = small_oracle["bvh"]
    b4 = oracle.bvh4_collapse(bvh)
    for masks, lut, mode in ((None, None, "none"), (small_oracle["masks6"], small_oracle["lut6"], "raw")):
        h = oracle.trace4(tris, bvh, b4, sel, mode=mode, R=6, masks=masks, origin_bound=small_oracle["origin_bound"],
                          stack_depth=True)
        assert h.deepest.max() >= 3  # the stack really grows
        for i in range(sel.shape[0]):
            st = _recursive_trace4(tris, bvh, b4, sel[i], masks, lut, 6, small_oracle["origin_bound"])
            assert st["best"] == h.prim[i]
            assert (st["box"], st["tri"]) == (h.box_tests[i], h.tri_tests[i]), i
            assert st["deep"] == h.deepest[i], i
            if mode == "raw":
                assert (st["mt"], st["mc"]) == (h.mask_tests[i], h.mask_culls[i]), i


def test_codebook_reference_counts(small_scene, small_oracle):
    """Tests per codebook entry (LUT mode): equal to the recursive formulation's own tally, summing
    to the per-ray mask tests, the same on one thread as on several, and zero for every entry no
    slot uses and for the full entries at the end of the codebook (never tested)."""
    tris, rays = small_scene
    sel = np.concatenate([_aimed_rays(tris, 150, 43), rays[::1024]])
    bvh = small_oracle["bvh"]
    b4 = oracle.bvh4_collapse(bvh)
    ob, lut = small_oracle["origin_bound"], small_oracle["lut6"]
    cb, idx = oracle.compress(small_oracle["masks6"], bvh.slot_boxes(), 6, 256)
    kw = dict(mode="lut", R=6, codebook=cb, cidx=idx, origin_bound=ob, codebook_refs=True)
    h = oracle.trace4(tris, bvh, b4, sel, nthreads=4, **kw)
    h1 = oracle.trace4(tris, bvh, b4, sel, nthreads=1, **kw)
    assert h.cb_refs.shape == (cb.shape[0],) and (h.cb_refs == h1.cb_refs).all()
    assert h.cb_refs.sum() == h.mask_tests.sum() > 0
    used = np.zeros(cb.shape[0], bool)
    used[idx] = True
    assert (h.cb_refs[~used] == 0).all()
    full = oracle.mask_bits(cb, 6).sum(-1) == 216
    assert full.any() and (h.cb_refs[full] == 0).all()
    tally = {}
    slot_masks = cb[idx]
    for i in range(sel.shape[0]):
        st = _recursive_trace4(tris, bvh, b4, sel[i], slot_masks, lut, 6, ob, cidx=idx)
        assert st["mt"] == h.mask_tests[i], i
        for k, v in st["refs"].items():
            tally[k] = tally.get(k, 0) + v
    want = np.zeros(cb.shape[0], np.uint64)
    for k, v in tally.items():
        want[k] = v
    assert (h.cb_refs.astype(np.uint64) == want).all()
    # raw mode has no codebook: nothing is counted
    assert oracle.trace4(tris, bvh, b4, sel[:50], mode="raw", R=6, masks=small_oracle["masks6"],
                         origin_bound=ob, codebook_refs=True).cb_refs is None


def test_mask_test_limit_recursive_and_monotone(small_scene, small_oracle):
    """Masks denser than the limit pass untested: the recursive formulation agrees on every count
    at several limits; hits never change; per ray, a lower limit (fewer tests) never gives fewer
    box or triangle tests; a limit below the sparsest mask tests nothing (plain counts)."""
    tris, rays = small_scene
    sel = np.concatenate([_aimed_rays(tris, 120, 41), rays[::2048]])
    bvh = small_oracle["bvh"]
    b4 = oracle.bvh4_collapse(bvh)
    masks, lut, ob = small_oracle["masks6"], small_oracle["lut6"], small_oracle["origin_bound"]
    pcs = oracle.mask_bits(masks, 6).sum(-1)
    plain = oracle.trace4(tris, bvh, b4, sel, origin_bound=ob)
    prev = None
    for limit in sorted({int(pcs.min()) - 1 or 1, int(np.percentile(pcs, 25)), int(np.median(pcs)), 215}):
        h = oracle.trace4(tris, bvh, b4, sel, mode="raw", R=6, masks=masks, origin_bound=ob, test_max=limit)
        assert (h.prim == plain.prim).all() and (h.t.view(np.uint32) == plain.t.view(np.uint32)).all()
        for i in range(0, sel.shape[0], 7):
            st = _recursive_trace4(tris, bvh, b4, sel[i], masks, lut, 6, ob, test_max=limit)
            assert (st["box"], st["tri"], st["mt"], st["mc"]) == \
                (h.box_tests[i], h.tri_tests[i], h.mask_tests[i], h.mask_culls[i]), (limit, i)
        if prev is not None:  # a higher limit tests a superset of masks
            assert (prev.box_tests >= h.box_tests).all() and (prev.tri_tests >= h.tri_tests).all()
            assert (prev.mask_tests <= h.mask_tests).all()
        prev = h
    # the default limit is R^3 - 1 (every mask but a full one)
    d = oracle.trace4(tris, bvh, b4, sel, mode="raw", R=6, masks=masks, origin_bound=ob)
    assert (d.box_tests == prev.box_tests).all() and (d.mask_tests == prev.mask_tests).all()
    low = oracle.trace4(tris, bvh, b4, sel, mode="raw", R=6, masks=masks, origin_bound=ob,
                        test_max=max(1, int(pcs.min()) - 1))
    if pcs.min() > 1:
        assert low.mask_tests.sum() == 0 and (low.box_tests == plain.box_tests).all()
