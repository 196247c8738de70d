"""GPU parity of the 4-wide BVH (Sect. 3.2.4 node: four child boxes, four
child masks) against the oracle: the collapsed nodes bit for bit, and per ray
hit id, t, box / triangle / mask counts, in every mask mode, culled and in
shadow mode (per binary slot counts), sorted and in every launch shape, plus
micro scenes and degenerate inputs."""
import numpy as np
import pytest

import oracle
from paper_2305_08343_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_2305_08343_amd import binding
    c = binding.Context(0)
    yield c
    c.close()


def _compare(dev, ora, masks=True):
    bad = np.flatnonzero((dev["prim"] != ora.prim) | (dev["t"].view(np.uint32) != ora.t.view(np.uint32)) |
                         (dev["box_tests"] != ora.box_tests) | (dev["tri_tests"] != ora.tri_tests))
    assert bad.size == 0, f"{bad.size} rays differ, first {bad[:5]}"
    if masks:
        assert (dev["mask_tests"] == ora.mask_tests).all() and (dev["mask_culls"] == ora.mask_culls).all()


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


def _kw(small_oracle, mode, R, K):
    bvh = small_oracle["bvh"]
    kw = dict(origin_bound=small_oracle["origin_bound"])
    if mode == "raw":
        kw.update(mode="raw", R=R, masks=small_oracle[f"masks{R}"])
    elif mode == "lut":
        cb, idx = oracle.compress(small_oracle[f"masks{R}"], bvh.slot_boxes(), R, K)
        kw.update(mode="lut", R=R, codebook=cb, cidx=idx)
    return kw


def test_collapse_matches_oracle(ctx, small_scene, small_oracle):
    from paper_2305_08343_amd import binding
    tris, _ = small_scene
    ob4 = oracle.bvh4_collapse(small_oracle["bvh"])
    for mode in ("none", "raw", "lut"):
        print(f"[gpu-bvh4] collapse export, mode {mode}", flush=True)
        s = binding.Scene(ctx, tris, R=6, mode=mode, K=4096, width=4)
        assert s.info["width"] == 4 and s.info["n_nodes"] == ob4.n4 and s.info["node_bytes"] == 128
        e = s.export4()
        s.close()
        assert (e["box4"].view(np.uint32) == ob4.box4.view(np.uint32)).all()
        assert (e["ref4"] == ob4.ref4).all() and (e["src4"] == ob4.src4).all()


@pytest.mark.parametrize("mode,R,K", [("none", 6, 0), ("raw", 6, 0), ("raw", 4, 0), ("lut", 6, 4096),
                                      ("lut", 6, 256), ("lut", 4, 256), ("lut", 4, 4096)])
def test_trace_bit_exact(ctx, small_scene, small_oracle, mode, R, K):
    import torch
    from paper_2305_08343_amd import binding
    tris, rays = small_scene
    rays = np.concatenate([rays, _aimed(tris, 30011, 41)])
    bvh = small_oracle["bvh"]
    b4 = oracle.bvh4_collapse(bvh)
    kw = _kw(small_oracle, mode, R, K)
    print(f"[gpu-bvh4] trace {mode} R={R} K={K}", flush=True)
    s = binding.Scene(ctx, tris, R=R, mode=mode, K=K or 4096, width=4)
    try:
        # LUT mode: codebook from LDS (when it fits) and from global memory
        for cbg in ((0, 1) if mode == "lut" else (0,)):
            ctx.set_tune(codebook=cbg)
            for cull in (True, False):
                _compare(s.trace(rays, cull=cull).numpy(), oracle.trace4(tris, bvh, b4, rays, cull=cull, **kw))
    finally:
        ctx.set_tune()
    if mode != "none":
        fp = torch.zeros(2 * bvh.n_inner, dtype=torch.int32, device="cuda:0")
        dev = s.trace(rays, cull=False, shadow=True, slot_fp=fp).numpy()
        ora = oracle.trace4(tris, bvh, b4, rays, cull=False, shadow=True, **kw)
        _compare(dev, ora)
        assert (fp.cpu().numpy().view(np.uint32) == ora.slot_fp).all() and ora.slot_fp.sum() > 0
    s.close()


@pytest.mark.parametrize("seed", range(16))
def test_micro_scenes(ctx, seed):
    from paper_2305_08343_amd import binding
    n = 1 + (seed * 13) % 64
    tris = scenes.micro_scene(seed, n)
    rays = np.concatenate([_aimed(tris, 300, seed), scenes.random_rays(100, seed)])
    bvh = oracle.bvh_build(tris)
    b4 = oracle.bvh4_collapse(bvh)
    ob, delta = oracle.default_bounds(tris)
    print(f"[gpu-bvh4] micro scene {seed} ({n} tris)", flush=True)
    for R in (4, 6):
        s = binding.Scene(ctx, tris, R=R, mode="raw", width=4)
        masks = oracle.object_masks(tris, bvh, R, delta)
        _compare(s.trace(rays).numpy(), oracle.trace4(tris, bvh, b4, rays, mode="raw", R=R, masks=masks,
                                                      origin_bound=ob))
        s.close()


def test_too_many_triangles_for_4_wide_rejected_before_any_read(ctx):
    import ctypes as C
    import torch
    from paper_2305_08343_amd import binding
    print("[gpu-bvh4] 2^28 triangles rejected", flush=True)
    lib = binding.load()
    p = binding.sc_build_params()
    lib.sc_build_params_default(C.byref(p))
    p.width = 4
    dummy = torch.zeros(9, dtype=torch.float32, device="cuda:0")  # never read: the count is checked first
    h = C.c_void_p()
    assert lib.sc_scene_build(ctx.handle, C.c_void_p(dummy.data_ptr()), 1 << 28, C.byref(p), None,
                              C.byref(h)) == 1
    assert b"2^28" in lib.sc_last_error() and not h.value


def test_degenerate_inputs(ctx, small_scene):
    from paper_2305_08343_amd import binding
    print("[gpu-bvh4] empty scene, single leaf, invalid rays", flush=True)
    rays = scenes.random_rays(1000, 3)
    s = binding.Scene(ctx, np.zeros((0, 3, 3), np.float32), mode="raw", width=4)
    d = s.trace(rays).numpy()
    s.close()
    assert (d["prim"] == oracle.NO_HIT).all() and (d["box_tests"] == 0).all()
    t = scenes.micro_scene(2, 3)
    bvh = oracle.bvh_build(t)
    s = binding.Scene(ctx, t, mode="raw", width=4)
    assert s.info["n_nodes"] == 0
    _compare(s.trace(rays).numpy(), oracle.trace4(t, bvh, oracle.bvh4_collapse(bvh), rays), masks=False)
    s.close()
    tris, _ = small_scene
    bad = rays.copy()
    bad[::3, 4:7] = 0.0
    bad[1::3, 0] = np.nan
    s = binding.Scene(ctx, tris, mode="raw", width=4)
    d = s.trace(bad).numpy()
    s.close()
    assert (d["box_tests"][::3] == 0).all() and (d["box_tests"][1::3] == 0).all()
    with pytest.raises(binding.SubcullError):
        binding.Scene(ctx, tris, mode="sparse", placement=np.ones(2, np.uint8), width=4)


def test_sorted_and_every_launch_shape(ctx, small_scene, small_oracle):
    from paper_2305_08343_amd import binding
    tris, rays = small_scene
    rays = np.concatenate([rays, _aimed(tris, 20000, 43)])
    bvh = small_oracle["bvh"]
    b4 = oracle.bvh4_collapse(bvh)
    ora = oracle.trace4(tris, bvh, b4, rays, **_kw(small_oracle, "raw", 6, 0))
    s = binding.Scene(ctx, tris, R=6, mode="raw", width=4)
    try:
        for block, stack in ((256, 8), (128, 8), (256, 12), (256, 4), (128, 16)):
            for chunk, parts, waves, sort, gather, refill in ((1, 8, 0, 0, 0, 1), (3, 1, 2, 1, 64, 64),
                                                              (2, 8, 5, 1, 8, 24)):
                print(f"[gpu-bvh4] tune {block} {stack} {chunk} {parts} {waves} {sort} {gather} {refill}",
                      flush=True)
                ctx.set_tune(block, stack, chunk, parts, waves, sort, 0, gather, refill)
                _compare(s.trace(rays).numpy(), ora)
    finally:
        ctx.set_tune()
        s.close()


def test_batches_take_4_wide_scenes(ctx, small_scene):
    """A 4-wide scene in a batched launch (graph and direct) gives its single-scene results; a
    batch mixing it with a binary scene is refused."""
    import torch
    from paper_2305_08343_amd import binding
    tris, rays = small_scene
    s = binding.Scene(ctx, tris, R=6, mode="raw", width=4)
    s2 = binding.Scene(ctx, tris, R=6, mode="raw", width=2)
    rd = torch.from_numpy(rays[:5000]).cuda()
    single = s.trace(rd).numpy()
    for graph in (True, False):
        b = binding.Batch(ctx, [(s, rd)], graph=graph)
        b.launch()
        torch.cuda.synchronize()
        got = b.results(0).numpy()
        for f in ("prim", "box_tests", "tri_tests", "mask_tests", "mask_culls"):
            assert (got[f] == single[f]).all(), (graph, f)
        b.close()
    with pytest.raises(binding.SubcullError):
        binding.Batch(ctx, [(s, rd), (s2, rd)], graph=False).launch()
    s.close()
    s2.close()


def test_features_of_4_wide_scene_are_the_binary_slot_features(ctx, small_scene):
    from paper_2305_08343_amd import binding
    tris, _ = small_scene
    print("[gpu-bvh4] slot features of a 4-wide scene", flush=True)
    for mode in ("raw", "lut"):
        s2 = binding.Scene(ctx, tris, R=6, mode=mode, width=2)
        s4 = binding.Scene(ctx, tris, R=6, mode=mode, width=4)
        f2, f4 = s2.features().cpu().numpy(), s4.features().cpu().numpy()
        s2.close()
        s4.close()
        assert (f2.view(np.uint32) == f4.view(np.uint32)).all()


def test_negative_zero_direction_on_a_box_plane_keeps_the_hit(ctx):
    """Both node widths keep a box hit for a ray with a -0 direction component
    that starts on the box's plane (near/far bounds chosen by the direction's
    sign), as the oracle and brute force do."""
    from paper_2305_08343_amd import binding
    tri = np.array([[[0.5, 0.4, 0.5], [0.5, 0.6, 0.5], [0.7, 0.5, 0.5]]], np.float32)
    far = np.array([[[5.0 + k, 5.0, 5.0], [5.2 + k, 5.0, 5.0], [5.0 + k, 5.2, 5.1]] for k in range(8)], np.float32)
    tris = np.concatenate([tri, far])
    rays = np.array([[0.5, 0.5, 0.0, 0.0, -0.0, 0.0, 1.0, np.inf],
                     [0.5, 0.5, 0.0, 0.0, 0.0, 0.0, 1.0, np.inf]], np.float32)
    bvh = oracle.bvh_build(tris)
    for width in (2, 4):
        print(f"[gpu-bvh4] -0 direction on a box plane, width {width}", flush=True)
        s = binding.Scene(ctx, tris, R=6, mode="raw", width=width)
        dev = s.trace(rays).numpy()
        s.close()
        assert (dev["prim"] == 0).all()
        ora = oracle.trace(tris, bvh, rays) if width == 2 else oracle.trace4(tris, bvh, oracle.bvh4_collapse(bvh), rays)
        assert (dev["t"].view(np.uint32) == ora.t.view(np.uint32)).all()
        assert (dev["box_tests"] == ora.box_tests).all()


@pytest.mark.parametrize("width,mode,R,K,bits,quant", [
    (2, "raw", 6, 4096, False, False), (2, "lut", 6, 256, False, False), (2, "raw", 4, 4096, False, False),
    (4, "raw", 6, 4096, False, False), (4, "raw", 4, 4096, False, True), (4, "lut", 6, 4096, True, False),
    (4, "lut", 6, 4096, True, True), (4, "lut", 4, 256, False, False)])
def test_mask_test_limit_bit_exact(ctx, small_scene, small_oracle, width, mode, R, K, bits, quant):
    """Masks (raw, or the codebook entry a slot points to) with more set bits than the build's
    limit pass untested: every count equals the oracle's at the same limit, hits equal those of
    plain traversal."""
    from paper_2305_08343_amd import binding
    tris, rays = small_scene
    rays = np.concatenate([rays[::3], _aimed(tris, 20011, 61)])
    bvh = small_oracle["bvh"]
    b4 = oracle.bvh4_collapse(bvh) if width == 4 else None
    if quant:
        b4 = oracle.decoded_bvh4(b4, oracle.quantise4(b4))
        bvh = oracle.with_slot_boxes(bvh, b4)
    masks = oracle.object_masks(tris, bvh, R, small_oracle["delta"])
    kw = dict(origin_bound=small_oracle["origin_bound"], mode=mode, R=R)
    if mode == "raw":
        kw["masks"] = masks
    else:
        cb, idx = oracle.compress(masks, bvh.slot_boxes(), R, K)
        kw.update(codebook=cb, cidx=idx)
    for limit in (R ** 3 // 4, R ** 3 // 2):
        print(f"[gpu-bvh4] test limit {limit}: width {width} {mode} R={R} K={K} bits={bits} q={quant}", flush=True)
        s = binding.Scene(ctx, tris, R=R, mode=mode, K=K, width=width, bit_table=bits, quantise=quant,
                          mask_test_max=limit)
        assert s.info["mask_test_max"] == limit
        dev = s.trace(rays).numpy()
        s.close()
        ora = oracle.trace4(tris, bvh, b4, rays, test_max=limit, **kw) if width == 4 else \
            oracle.trace(tris, bvh, rays, test_max=limit, **kw)
        _compare(dev, ora)
        assert (dev["t"].view(np.uint32) == ora.t.view(np.uint32)).all()
        assert ora.mask_tests.sum() > 0
    with pytest.raises(binding.SubcullError):
        binding.Scene(ctx, tris, R=R, mode=mode, K=K, width=width, mask_test_max=R ** 3)
