"""Batched traversal (one persistent launch over many scenes, optionally
replayed from a HIP graph): every item's results equal the single-scene
traversal of that item, bit for bit, which in turn equals the oracle."""
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


def _scene_set(n_scenes=9):
    """Uneven sizes and kinds, plus an empty scene and a single-leaf scene."""
    out = []
    for i in range(n_scenes):
        kind = i % 3
        if kind == 0:
            t = scenes.strands_helical(300 + i, 40 + 60 * i, 12, 1e-3, 5e-3, 0.25, (0.05,) * 3, (0.95,) * 3)
        elif kind == 1:
            t = scenes.thin_quads(300 + i, 200 + 400 * i, 0.05, 1e-3)
        else:
            t = scenes.isotropic_tris(300 + i, 300 + 700 * i, 0.03)
        n_rays = [5000, 0, 777, 20000, 64, 3000, 12345, 1, 9000][i % 9]
        r = np.concatenate([scenes.pinhole_rays(max(1, int(np.sqrt(n_rays // 2 + 1))), max(1, int(np.sqrt(n_rays // 2 + 1)))),
                            scenes.random_rays(n_rays, 400 + i)])[:n_rays]
        out.append((t, r))
    out.append((np.zeros((0, 3, 3), np.float32), scenes.random_rays(300, 7)))
    out.append((scenes.micro_scene(2, 3), scenes.random_rays(500, 8)))
    return out


def _same(a, b):
    return (a.hits.cpu().numpy() == b.hits.cpu().numpy()).all() and \
        (a.extra.cpu().numpy() == b.extra.cpu().numpy()).all()


@pytest.mark.parametrize("mode,R,K", [("raw", 6, 4096), ("none", 6, 4096), ("raw", 4, 4096),
                                      ("lut", 6, 256), ("lut", 4, 256)])
def test_batch_equals_single_scene_traces(ctx, mode, R, K):
    import torch
    from paper_2305_08343_amd import binding
    print(f"[gpu] batch mode={mode} R={R} K={K}", flush=True)
    items = _scene_set()
    built = [binding.Scene(ctx, t, R=R, mode=mode, K=K) for t, _ in items]
    singles = [s.trace(r) for s, (_, r) in zip(built, items)]
    for graph in (False, True):
        b = binding.Batch(ctx, [(s, r) for s, (_, r) in zip(built, items)], graph=graph)
        b.launch()
        torch.cuda.synchronize()
        for k in range(len(items)):
            assert _same(b.results(k), singles[k]), (graph, k)
        b.close()
    # one item checked against the oracle as well
    t, r = items[3]
    bvh = oracle.bvh_build(t)
    ob, delta = oracle.default_bounds(t)
    kw = dict(origin_bound=ob)
    if mode == "raw":
        kw.update(mode="raw", R=R, masks=oracle.object_masks(t, bvh, R, delta))
    elif mode == "lut":
        cb, idx = oracle.compress(oracle.object_masks(t, bvh, R, delta), bvh.slot_boxes(), R, K)
        kw.update(mode="lut", R=R, codebook=cb, cidx=idx)
    ora = oracle.trace(t, bvh, r, **kw)
    d = singles[3].numpy()
    assert (d["prim"] == ora.prim).all() and (d["box_tests"] == ora.box_tests).all()
    assert (d["mask_tests"] == ora.mask_tests).all()
    for s in built:
        s.close()


def test_graph_replays_with_eager_work_between(ctx):
    import torch
    from paper_2305_08343_amd import binding
    print("[gpu] graph replays", flush=True)
    items = _scene_set(6)
    built = [binding.Scene(ctx, t, R=6, mode="raw") for t, _ in items]
    b = binding.Batch(ctx, [(s, r) for s, (_, r) in zip(built, items)], graph=True)
    ref = [s.trace(b.rays[k]) for k, s in enumerate(built)]
    ref_np = [(x.hits.cpu().numpy().copy(), x.extra.cpu().numpy().copy()) for x in ref]
    for rep in range(4):
        for k in range(len(items)):  # scribble over the outputs between replays
            b.hits[k].fill_(-7)
        junk = torch.randn(1 << 20, device="cuda") * 3.0  # eager work on the same stream
        _ = built[rep % len(built)].trace(b.rays[rep % len(built)])
        b.launch()
        junk.sum().item()
        torch.cuda.synchronize()
        for k in range(len(items)):
            n = b.rays[k].shape[0]
            assert (b.hits[k][:n].cpu().numpy() == ref_np[k][0]).all(), (rep, k)
            assert (b.extra[k][:n].cpu().numpy() == ref_np[k][1]).all(), (rep, k)
    # new ray contents in the bound buffers are picked up by the next replay
    k = 3
    new = torch.from_numpy(scenes.random_rays(b.rays[k].shape[0], 99)).cuda()
    b.rays[k].copy_(new)
    b.launch()
    torch.cuda.synchronize()
    assert _same(b.results(k), built[k].trace(new))
    b.close()
    for s in built:
        s.close()


def test_batch_rejects_mixed_modes(ctx):
    from paper_2305_08343_amd import binding
    t = scenes.scene_small(0)
    a = binding.Scene(ctx, t, R=6, mode="raw")
    c = binding.Scene(ctx, t, R=4, mode="raw")
    r = scenes.rays_small(32)
    with pytest.raises(binding.SubcullError) as e:
        binding.Batch(ctx, [(a, r), (c, r)], graph=False).launch()
    assert e.value.status == 1
    a.close()
    c.close()


@pytest.mark.parametrize("mode,R,K,quant", [("none", 6, 4096, True), ("raw", 4, 4096, True), ("raw", 6, 4096, False),
                                            ("lut", 6, 4096, False), ("lut", 4, 256, True), ("none", 6, 4096, False)])
def test_batch_4_wide_equals_single_scene_traces(ctx, mode, R, K, quant):
    """4-wide nodes (float or quantised child boxes) in one persistent launch, direct and replayed
    from a HIP graph: every item equals its single-scene trace (in which a codebook that fits is
    read from LDS, in the batch from global memory), which equals the oracle's 4-wide traversal."""
    import torch
    from paper_2305_08343_amd import binding
    print(f"[gpu] 4-wide batch mode={mode} R={R} K={K} quantised={quant}", flush=True)
    items = _scene_set()
    built = [binding.Scene(ctx, t, R=R, mode=mode, K=K, width=4, quantise=quant) for t, _ in items]
    singles = [s.trace(r) for s, (_, r) in zip(built, items)]
    for graph in (False, True):
        b = binding.Batch(ctx, [(s, r) for s, (_, r) in zip(built, items)], graph=graph)
        b.launch()
        b.launch()
        torch.cuda.synchronize()
        for k in range(len(items)):
            assert _same(b.results(k), singles[k]), (graph, k)
        b.close()
    for k in (3, 8):  # a larger scene and the 1-ray scene against the oracle
        t, r = items[k]
        bvh = oracle.bvh_build(t)
        b4 = oracle.bvh4_collapse(bvh)
        if quant:
            b4 = oracle.decoded_bvh4(b4, oracle.quantise4(b4))
            bvh = oracle.with_slot_boxes(bvh, b4)
        ob, delta = oracle.default_bounds(t)
        kw = dict(origin_bound=ob)
        if mode == "raw":
            kw.update(mode="raw", R=R, masks=oracle.object_masks(t, bvh, R, delta))
        elif mode == "lut":
            cb, idx = oracle.compress(oracle.object_masks(t, bvh, R, delta), bvh.slot_boxes(), R, K)
            kw.update(mode="lut", R=R, codebook=cb, cidx=idx)
        ora = oracle.trace4(t, bvh, b4, r, **kw)
        d = singles[k].numpy()
        assert (d["prim"] == ora.prim).all() and (d["t"].view(np.uint32) == ora.t.view(np.uint32)).all()
        assert (d["box_tests"] == ora.box_tests).all() and (d["tri_tests"] == ora.tri_tests).all()
        assert (d["mask_tests"] == ora.mask_tests).all() and (d["mask_culls"] == ora.mask_culls).all()
    for s in built:
        s.close()


def test_batch_4_wide_shadow_counts_per_slot(ctx):
    """Shadow mode in a 4-wide batch adds would-be culls to each item's own per-slot counters,
    exactly as single-scene shadow traces do."""
    import torch
    from paper_2305_08343_amd import binding
    items = _scene_set(6)
    built = [binding.Scene(ctx, t, R=6, mode="raw", width=4) for t, _ in items]
    fps = [torch.zeros(max(2 * s.info["n_inner"], 1), dtype=torch.int32, device="cuda") for s in built]
    b = binding.Batch(ctx, [(s, r) for s, (_, r) in zip(built, items)], cull=False, shadow=True, graph=False,
                      slot_fp=fps)
    b.launch()
    torch.cuda.synchronize()
    for k, s in enumerate(built):
        ref = torch.zeros_like(fps[k])
        s.trace(items[k][1], cull=False, shadow=True, slot_fp=ref)
        torch.cuda.synchronize()
        assert torch.equal(ref, fps[k]), k
    assert sum(int(f.sum().item()) for f in fps) > 0
    b.close()
    for s in built:
        s.close()


def test_batch_rejects_mixed_widths(ctx):
    from paper_2305_08343_amd import binding
    t = scenes.scene_small(0)
    a = binding.Scene(ctx, t, R=6, mode="raw")
    c = binding.Scene(ctx, t, R=6, mode="raw", width=4)
    d = binding.Scene(ctx, t, R=6, mode="raw", width=4, quantise=True)
    r = scenes.rays_small(32)
    for pair in ((a, c), (c, d)):
        with pytest.raises(binding.SubcullError) as e:
            binding.Batch(ctx, [(pair[0], r), (pair[1], r)], graph=False).launch()
        assert e.value.status == 1
    for s in (a, c, d):
        s.close()


@pytest.mark.parametrize("width,mode,R,quant", [(2, "raw", 6, False), (4, "raw", 4, True), (4, "lut", 6, False)])
def test_sorted_batch_equals_single_scene_traces(ctx, width, mode, R, quant):
    """Rays taken in (item, Morton code of the origin) order, in one launch and from a graph whose
    replays re-order the rays' current contents: every result equals the single-scene trace."""
    import torch
    from paper_2305_08343_amd import binding
    print(f"[gpu] sorted batch width={width} mode={mode} R={R} quantised={quant}", flush=True)
    items = _scene_set()
    built = [binding.Scene(ctx, t, R=R, mode=mode, K=256, width=width, quantise=quant) for t, _ in items]
    singles = [s.trace(r) for s, (_, r) in zip(built, items)]
    for graph in (False, True):
        b = binding.Batch(ctx, [(s, r) for s, (_, r) in zip(built, items)], graph=graph, sort=True)
        b.launch()
        torch.cuda.synchronize()
        for k in range(len(items)):
            assert _same(b.results(k), singles[k]), (graph, k)
        # new ray contents: the next launch orders and traces those
        k = 3
        new = torch.from_numpy(scenes.random_rays(b.rays[k].shape[0], 1234)).cuda()
        b.rays[k].copy_(new)
        b.launch()
        torch.cuda.synchronize()
        assert _same(b.results(k), built[k].trace(new)), graph
        assert _same(b.results(0), singles[0]), graph
        b.rays[k].copy_(torch.from_numpy(items[k][1]).cuda())
        b.close()
    for s in built:
        s.close()


def test_sorted_batch_launch_shape_and_item_limit(ctx):
    """The launch shape's sort applies to batches too; a sorted batch of more than 256 items is
    refused (the item index takes the key's top 8 bits)."""
    import torch
    from paper_2305_08343_amd import binding
    items = _scene_set(6)
    built = [binding.Scene(ctx, t, R=6, mode="raw") for t, _ in items]
    singles = [s.trace(r) for s, (_, r) in zip(built, items)]
    t = ctx.get_tune()
    try:
        ctx.set_tune(t["block"], t["stack"], t["chunk"], t["parts"], t["waves"], 1, t["codebook"], t["gather"],
                     t["refill"])
        b = binding.Batch(ctx, [(s, r) for s, (_, r) in zip(built, items)], graph=False)
        b.launch()
        torch.cuda.synchronize()
        for k in range(len(items)):
            assert _same(b.results(k), singles[k]), k
        b.close()
        r = scenes.random_rays(8, 5)
        many = [(built[0], r)] * 257
        with pytest.raises(binding.SubcullError) as e:
            binding.Batch(ctx, many, graph=False).launch()
        assert e.value.status == 6
    finally:
        ctx.set_tune()
    for s in built:
        s.close()
