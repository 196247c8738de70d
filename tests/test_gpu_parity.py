"""GPU parity: every product of the HIP path against the oracle.

Bar (integer work bit-exact; the float32 hit distance is bit-exact too,
which is within the stated 1e-5 relative tolerance): ray-mask LUT, BVH
topology/boxes/permutation, object masks, codebook, Alg. 3 indices, and per
ray the hit id, t, box/triangle/mask test counts and mask culls. Sizes span
many 128-ray blocks with a ragged tail, plus the degenerate cases.
"""
import numpy as np
import pytest

import oracle
from paper_2305_08343_amd import scenes

pytestmark = pytest.mark.gpu
NO_HIT = 0xFFFFFFFF


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_2305_08343_amd import binding
    c = binding.Context(0)
    yield c
    c.close()


def _compare_hits(dev, ora, with_masks=True):
    bad = np.flatnonzero((dev["prim"] != ora.prim) |
                         (dev["t"].view(np.uint32) != ora.t.view(np.uint32)) |
                         (dev["box_tests"] != ora.box_tests) | (dev["tri_tests"] != ora.tri_tests))
    assert bad.size == 0, f"{bad.size} rays differ, first {bad[:5]}"
    if with_masks:
        assert (dev["mask_tests"] == ora.mask_tests).all()
        assert (dev["mask_culls"] == ora.mask_culls).all()


def _aimed(tris, n, seed):
    rng = np.random.default_rng(seed)
    lo, hi = tris.reshape(-1, 3).min(0), tris.reshape(-1, 3).max(0)
    c, ext = 0.5 * (lo + hi), np.maximum(hi - lo, 1e-3)
    o = c + (rng.random((n, 3)) - 0.5) * ext * 2.2
    t = rng.integers(0, tris.shape[0], n)
    w = rng.dirichlet([1, 1, 1], n)
    d = np.einsum("nk,nkj->nj", w, tris[t].astype(np.float64)) - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = np.zeros((n, 8), np.float32)
    r[:, :3], r[:, 4:7], r[:, 7] = o, d, np.inf
    return r


def _check_bvh(exp, ob):
    assert exp["cbox"].shape == ob.cbox.shape
    assert (exp["cbox"].view(np.uint32) == ob.cbox.view(np.uint32)).all()
    assert (exp["cref"] == ob.cref).all() and (exp["range"] == ob.range).all()
    assert (exp["perm"] == ob.perm).all()


@pytest.mark.parametrize("R", [4, 6])
def test_raymask_lut_bit_exact(ctx, R):
    print(f"[gpu] raymask LUT R={R}", flush=True)
    assert (ctx.raymask_lut(R) == oracle.raymask_lut(R)).all()


def test_small_scene_build_bit_exact(ctx, small_scene, small_oracle):
    from paper_2305_08343_amd import binding
    tris, _ = small_scene
    for R in (4, 6):
        print(f"[gpu] small scene build R={R}", flush=True)
        s = binding.Scene(ctx, tris, R=R, mode="raw")
        assert s.info["delta"] == np.float32(small_oracle["delta"])
        assert s.info["origin_bound"] == np.float32(small_oracle["origin_bound"])
        assert s.info["depth"] == small_oracle["bvh"].depth
        exp = s.export()
        _check_bvh(exp, small_oracle["bvh"])
        assert (exp["masks"] == small_oracle[f"masks{R}"]).all()
        s.close()


@pytest.mark.parametrize("mode,R,K", [("none", 6, 0), ("raw", 4, 0), ("raw", 6, 0),
                                      ("lut", 6, 256), ("lut", 6, 4096), ("lut", 4, 256)])
def test_small_scene_trace_bit_exact(ctx, small_scene, small_oracle, mode, R, K):
    from paper_2305_08343_amd import binding
    tris, rays = small_scene
    rays = np.concatenate([rays, _aimed(tris, 30001, 7)])  # ragged tail
    print(f"[gpu] small trace mode={mode} R={R} K={K} rays={rays.shape[0]}", flush=True)
    s = binding.Scene(ctx, tris, R=R, mode=mode, K=K or 4096)
    bvh = small_oracle["bvh"]
    kw = dict(origin_bound=small_oracle["origin_bound"])
    if mode == "raw":
        kw.update(mode="raw", R=R, masks=small_oracle[f"masks{R}"])
    elif mode == "lut":
        exp = s.export()
        cb, idx = oracle.compress(small_oracle[f"masks{R}"], bvh.slot_boxes(), R, K)
        assert (exp["codebook"] == cb).all()
        assert (exp["cidx"] == idx).all()
        kw.update(mode="lut", R=R, codebook=cb, cidx=idx)
    try:
        # LUT mode: codebook from LDS (when it fits) and from global memory
        for cbg in ((0, 1) if mode == "lut" else (0,)):
            ctx.set_tune(codebook=cbg)
            for cull in (True, False):
                ora = oracle.trace(tris, bvh, rays, cull=cull, **kw)
                dev = s.trace(rays, cull=cull).numpy()
                _compare_hits(dev, ora)
    finally:
        ctx.set_tune()
        s.close()


@pytest.mark.parametrize("R", [4, 6])
def test_sparse_placement_bit_exact(ctx, small_scene, small_oracle, R):
    from paper_2305_08343_amd import binding
    tris, rays = small_scene
    rays = np.concatenate([rays, _aimed(tris, 20000, 11)])
    bvh = small_oracle["bvh"]
    S = 2 * bvh.n_inner
    rng = np.random.default_rng(R)
    for frac in (0.0, 0.3, 1.0):
        placed = (rng.random(S) < frac).astype(np.uint8)
        print(f"[gpu] sparse R={R} placed fraction {frac}", flush=True)
        s = binding.Scene(ctx, tris, R=R, mode="sparse", placement=placed)
        dev = s.trace(rays).numpy()
        s.close()
        ora = oracle.trace(tris, bvh, rays, mode="sparse", R=R, masks=small_oracle[f"masks{R}"],
                           placed=placed, origin_bound=small_oracle["origin_bound"])
        _compare_hits(dev, ora)


def test_shadow_counts_bit_exact(ctx, small_scene, small_oracle):
    import torch
    from paper_2305_08343_amd import binding
    tris, rays = small_scene
    rays = np.concatenate([rays, _aimed(tris, 20000, 8)])
    print("[gpu] shadow-mode per-slot counts", flush=True)
    s = binding.Scene(ctx, tris, R=6, mode="raw")
    fp = torch.zeros(2 * s.info["n_inner"], dtype=torch.int32, device="cuda:0")
    dev = s.trace(rays, cull=False, shadow=True, slot_fp=fp).numpy()
    ora = oracle.trace(tris, small_oracle["bvh"], rays, mode="raw", R=6, masks=small_oracle["masks6"],
                       origin_bound=small_oracle["origin_bound"], cull=False, shadow=True)
    _compare_hits(dev, ora)
    assert (fp.cpu().numpy().view(np.uint32) == ora.slot_fp).all()
    assert ora.slot_fp.sum() > 0
    s.close()


def test_device_alg3_matches_oracle(ctx, small_oracle):
    rng = np.random.default_rng(3)
    for R, K in ((6, 4096), (6, 256), (4, 256), (4, 1024)):
        print(f"[gpu] Alg. 3 R={R} K={K}", flush=True)
        masks = small_oracle[f"masks{R}"]
        cb = oracle.codebook(masks, small_oracle["bvh"].slot_boxes(), R, K)
        req = oracle.req_luts(cb, R)
        bits = rng.random((5000, R ** 3)) < 0.1
        extra = np.zeros((5000, oracle.words_for(R)), np.uint64)
        for b in range(R ** 3):
            extra[:, b >> 6] |= bits[:, b].astype(np.uint64) << np.uint64(b & 63)
        q = np.concatenate([masks, extra])
        assert (ctx.compress_masks(R, cb, q) == oracle.alg3(q, req, K, R)).all()


@pytest.mark.parametrize("seed", range(24))
def test_micro_scenes_bit_exact(ctx, seed):
    from paper_2305_08343_amd import binding
    n = 1 + (seed * 11) % 64
    tris = scenes.micro_scene(seed, n)
    rays = np.concatenate([_aimed(tris, 257, seed), scenes.random_rays(63, seed)])
    print(f"[gpu] micro scene seed={seed} n={n}", flush=True)
    bvh = oracle.bvh_build(tris)
    ob, delta = oracle.default_bounds(tris)
    for mode, R in (("none", 6), ("raw", 4), ("raw", 6), ("lut", 6)):
        s = binding.Scene(ctx, tris, R=R, mode=mode, K=64)
        exp = s.export()
        _check_bvh(exp, bvh)
        kw = dict(origin_bound=ob)
        if mode != "none" and bvh.n_inner:
            m = oracle.object_masks(tris, bvh, R, delta)
            assert (exp["masks"] == m).all()
            if mode == "raw":
                kw.update(mode="raw", R=R, masks=m)
            else:
                cb, idx = oracle.compress(m, bvh.slot_boxes(), R, 64)
                assert (exp["codebook"] == cb).all() and (exp["cidx"] == idx).all()
                kw.update(mode="lut", R=R, codebook=cb, cidx=idx)
        _compare_hits(s.trace(rays).numpy(), oracle.trace(tris, bvh, rays, **kw))
        s.close()


@pytest.mark.parametrize("scene", ["lattice1", "lattice40", "segments"])
def test_codebook_selection_matches_oracle(ctx, scene):
    """Device codebook selection (importance sums per distinct mask in slot order, importance
    descending, ties by value) against the oracle: one mask shared by hundreds of slots, more
    distinct masks than K - 1 (lattice of 40 shapes: 94 at R = 4, 118 at R = 6), and the last
    chosen place falling among distinct masks tied at importance 0 (segments, R = 4, K = 64)."""
    from paper_2305_08343_amd import binding
    tris = scenes.segment_rows(0) if scene == "segments" else scenes.lattice_copies(int(scene[7:]))
    bvh = oracle.bvh_build(tris)
    _, delta = oracle.default_bounds(tris)
    for R in (4, 6):
        m = oracle.object_masks(tris, bvh, R, delta)
        for K in (64, 256, 4096):
            print(f"[gpu] codebook {scene} R={R} K={K} slots={m.shape[0]}", flush=True)
            s = binding.Scene(ctx, tris, R=R, mode="lut", K=K)
            exp = s.export()
            s.close()
            cb, idx = oracle.compress(m, bvh.slot_boxes(), R, K)
            assert (exp["masks"] == m).all()
            assert (exp["codebook"] == cb).all()
            assert (exp["cidx"] == idx).all()


def test_degenerate_inputs(ctx, small_scene):
    import torch
    from paper_2305_08343_amd import binding
    tris, rays = small_scene
    print("[gpu] degenerate inputs", flush=True)
    # empty scene: every ray misses with zero counts
    s = binding.Scene(ctx, np.zeros((0, 3, 3), np.float32), mode="raw")
    d = s.trace(rays[:1000]).numpy()
    assert (d["prim"] == NO_HIT).all() and np.isinf(d["t"]).all() and (d["box_tests"] == 0).all()
    s.close()
    # single leaf (no inner node)
    t3 = scenes.micro_scene(2, 3)
    s = binding.Scene(ctx, t3, mode="raw")
    r = _aimed(t3, 500, 1)
    ora = oracle.trace(t3, oracle.bvh_build(t3), r)
    _compare_hits(s.trace(r).numpy(), ora)
    s.close()
    # zero rays, one ray, invalid rays
    s = binding.Scene(ctx, tris, mode="raw")
    res = s.trace(rays[:0])
    assert res.hits.shape[0] == 0
    one = s.trace(rays[:1]).numpy()
    assert one["box_tests"].shape == (1,)
    bad = np.repeat(rays[:1], 6, 0)
    bad[0, 0] = np.nan
    bad[1, 4:7] = 0
    bad[2, 3], bad[2, 7] = 2.0, 1.0
    bad[3, 7] = np.nan
    bad[4, 5] = np.inf
    bad[5, 3] = -np.inf
    d = s.trace(bad).numpy()
    assert (d["prim"] == NO_HIT).all() and (d["box_tests"] == 0).all() and (d["tri_tests"] == 0).all()
    # a failed call leaves the scene usable
    with pytest.raises(binding.SubcullError):
        binding.load()
        from paper_2305_08343_amd.binding import _check, load
        _check(load().sc_trace(s.handle, None, 5, 1, None, None, None, None), "sc_trace")
    d2 = s.trace(rays[:300]).numpy()
    assert d2["box_tests"].sum() > 0
    # depth cap is reported, non-finite vertices are rejected
    with pytest.raises(binding.SubcullError) as e:
        binding.Scene(ctx, tris, depth_cap=3)
    assert e.value.status == 4
    t_bad = tris.copy()
    t_bad[5, 1, 2] = np.inf
    with pytest.raises(binding.SubcullError) as e:
        binding.Scene(ctx, t_bad)
    assert e.value.status == 1
    s.close()
    torch.cuda.synchronize()


def test_long_runs_of_invalid_rays(ctx, small_scene, small_oracle):
    """Whole chunks of rays that finish at once must not end a wave early."""
    from paper_2305_08343_amd import binding
    tris, rays = small_scene
    print("[gpu] runs of invalid rays", flush=True)
    r = np.concatenate([_aimed(tris, 3000, 9), rays[:3000]])
    bad = np.zeros(len(r), bool)
    bad[100:1400] = True          # > 2 chunks of consecutive invalid rays
    bad[2000:2070] = True
    bad[4500::7] = True
    r[bad, 4:7] = 0.0
    s = binding.Scene(ctx, tris, mode="raw")
    dev = s.trace(r).numpy()
    ora = oracle.trace(tris, small_oracle["bvh"], r, mode="raw", R=6, masks=small_oracle["masks6"],
                       origin_bound=small_oracle["origin_bound"])
    _compare_hits(dev, ora)
    assert (dev["box_tests"][bad] == 0).all() and (dev["box_tests"][~bad] > 0).any()
    s.close()


def test_every_launch_shape_gives_the_same_results(ctx, small_scene, small_oracle):
    from paper_2305_08343_amd import binding
    tris, rays = small_scene
    r = np.concatenate([rays, _aimed(tris, 20000, 10)])
    ora = oracle.trace(tris, small_oracle["bvh"], r, mode="raw", R=6, masks=small_oracle["masks6"],
                       origin_bound=small_oracle["origin_bound"])
    ora4 = oracle.trace(tris, small_oracle["bvh"], r, mode="raw", R=4, masks=small_oracle["masks4"],
                        origin_bound=small_oracle["origin_bound"])
    s6 = binding.Scene(ctx, tris, R=6, mode="raw")
    s4 = binding.Scene(ctx, tris, R=4, mode="raw")
    try:
        for block, stack in ((256, 8), (128, 8), (256, 12), (256, 4), (128, 16)):
            for chunk, parts, waves, sort, gather, refill in ((1, 8, 0, 0, 16, 16), (3, 1, 2, 1, 0, 64),
                                                              (64, 5, 0, 0, 64, 1), (2, 8, 5, 1, 8, 0)):
                print(f"[gpu] tune block={block} stack={stack} chunk={chunk} parts={parts} waves={waves} "
                      f"sort={sort} gather={gather} refill={refill}", flush=True)
                ctx.set_tune(block, stack, chunk, parts, waves, sort, 0, gather, refill)
                _compare_hits(s6.trace(r).numpy(), ora)
                _compare_hits(s4.trace(r).numpy(), ora4)
        with pytest.raises(binding.SubcullError):
            ctx.set_tune(64, 8, 1)
        with pytest.raises(binding.SubcullError):
            ctx.set_tune(256, 8, 1, 8, 9)
        with pytest.raises(binding.SubcullError):
            ctx.set_tune(256, 8, 1, 8, 0, 2)
        with pytest.raises(binding.SubcullError):
            ctx.set_tune(256, 8, 1, 8, 0, 0, 2)
        with pytest.raises(binding.SubcullError):
            ctx.set_tune(256, 8, 1, 8, 0, 0, 0, 65)
        with pytest.raises(binding.SubcullError):
            ctx.set_tune(256, 8, 1, 8, 0, 0, 0, 16, 65)
    finally:
        ctx.set_tune(256, 8, 1, 8)
        s6.close()
        s4.close()


def test_repeat_trace_is_deterministic(ctx, small_scene):
    from paper_2305_08343_amd import binding
    tris, rays = small_scene
    print("[gpu] determinism", flush=True)
    s = binding.Scene(ctx, tris, mode="lut", K=256)
    a = s.trace(rays).hits.cpu().numpy()
    b = s.trace(rays).hits.cpu().numpy()
    assert (a == b).all()
    s.close()


def _morton_keys_f32(rays, tris):
    """Morton code of each origin, 256 cells per axis of the vertex bounds,
    evaluated in float32 in the documented order: u = (p - lo) * (256 / (hi - lo))."""
    v = tris.reshape(-1, 3)
    lo, hi = v.min(0).astype(np.float32), v.max(0).astype(np.float32)
    ext = (hi - lo).astype(np.float32)
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        sc = np.where((ext > 0) & np.isfinite(np.float32(256) / ext), np.float32(256) / ext, np.float32(0))
        u = (rays[:, 0:3].astype(np.float32) - lo) * sc.astype(np.float32)
    finite = np.clip(np.nan_to_num(u, nan=0.0, posinf=255.0, neginf=0.0), 0.0, 255.0)
    cell = np.where(~(u > 0), 0, np.where(u >= 255, 255, finite.astype(np.int64)))
    key = np.zeros(rays.shape[0], np.int64)
    for b in range(8):  # bit b of x, y, z -> bits 3b+2, 3b+1, 3b
        for j, sh in ((0, 2), (1, 1), (2, 0)):
            key |= ((cell[:, j] >> b) & 1) << (3 * b + sh)
    return key


@pytest.mark.parametrize("n", [1, 4095, 4096, 3 * 4096 + 77, 300_001])
def test_ray_order_is_the_stable_morton_order(ctx, small_scene, n):
    from paper_2305_08343_amd import binding
    tris, _ = small_scene
    rng = np.random.default_rng(n)
    rays = scenes.random_rays(n, n + 5, lo=(-0.2, -0.2, -0.2), hi=(1.2, 1.2, 1.2))
    if n > 10:
        rays[: n // 7] = rays[0]            # many equal keys: stability decides their order
        rays[3, 0] = np.nan                 # NaN origin -> cell 0
        rays[5, :3] = (1e30, -1e30, 0.5)    # clamped
    rays = rays[rng.permutation(n)]
    print(f"[gpu] ray order n={n}", flush=True)
    s = binding.Scene(ctx, tris, R=6, mode="none")
    order = s.ray_order(rays).cpu().numpy()
    s.close()
    expect = np.argsort(_morton_keys_f32(rays, tris), kind="stable")
    assert (order == expect).all()


@pytest.mark.parametrize("mode,R,K", [("none", 6, 0), ("raw", 6, 0), ("raw", 4, 0), ("lut", 6, 4096),
                                      ("lut", 4, 256), ("sparse", 6, 0)])
def test_sorted_trace_matches_oracle(ctx, small_scene, small_oracle, mode, R, K):
    import torch
    from paper_2305_08343_amd import binding
    tris, rays = small_scene
    rays = np.concatenate([rays, _aimed(tris, 30011, 21)])
    bvh = small_oracle["bvh"]
    kw = dict(origin_bound=small_oracle["origin_bound"])
    placed = None
    if mode == "sparse":
        placed = (np.random.default_rng(5).random(2 * bvh.n_inner) < 0.4).astype(np.uint8)
        kw.update(mode="sparse", R=R, masks=small_oracle[f"masks{R}"], placed=placed)
    elif mode == "raw":
        kw.update(mode="raw", R=R, masks=small_oracle[f"masks{R}"])
    elif mode == "lut":
        cb, idx = oracle.compress(small_oracle[f"masks{R}"], bvh.slot_boxes(), R, K)
        kw.update(mode="lut", R=R, codebook=cb, cidx=idx)
    print(f"[gpu] sorted trace {mode} R={R} K={K}", flush=True)
    s = binding.Scene(ctx, tris, R=R, mode=mode, K=K or 4096, placement=placed)
    fp = torch.zeros(max(1, 2 * s.info["n_inner"]), dtype=torch.int32, device="cuda:0")
    dev = s.trace(rays, sort=True).numpy()
    shadow = s.trace(rays, sort=True, cull=False, shadow=True, slot_fp=fp).numpy()
    s.close()
    _compare_hits(dev, oracle.trace(tris, bvh, rays, **kw))
    ora_sh = oracle.trace(tris, bvh, rays, cull=False, shadow=True, **kw)
    _compare_hits(shadow, ora_sh)
    if mode != "none":
        assert (fp.cpu().numpy()[:2 * bvh.n_inner].view(np.uint32) == ora_sh.slot_fp).all()
