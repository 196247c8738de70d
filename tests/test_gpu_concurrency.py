"""Two host threads on one fresh context: each builds a scene (the first use
builds the context's ray-mask tables) and traces it three times on its own
stream, one the binary BVH and one the 4-wide BVH, at the same time. Every
result must equal the oracle's: the shared tables are complete before any
stream uses them, and the launcher's per-kernel occupancy cache is filled
once for both threads."""
import threading

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _same(d, o):
    return bool((d["prim"] == o.prim).all() and (d["t"].view(np.uint32) == o.t.view(np.uint32)).all()
                and (d["box_tests"] == o.box_tests).all() and (d["tri_tests"] == o.tri_tests).all()
                and (d["mask_tests"] == o.mask_tests).all() and (d["mask_culls"] == o.mask_culls).all())


@pytest.mark.timeout(300)
def test_two_threads_two_streams_one_fresh_context():
    import torch
    assert torch.cuda.is_available()
    from paper_2305_08343_amd import binding, scenes
    tris = scenes.scene_small(0)
    rays = scenes.rays_small(128)
    ctx = binding.Context(0)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    results, errors = [None, None], []

    def work(i):
        try:
            with torch.cuda.stream(streams[i]):
                sc = binding.Scene(ctx, tris, R=6, mode="raw", width=2 if i == 0 else 4, stream=streams[i])
                rd = torch.from_numpy(rays).cuda()
                outs = [sc.trace(rd, stream=streams[i]) for _ in range(3)]
                streams[i].synchronize()
                results[i] = [o.numpy() for o in outs]
                sc.close()
        except Exception as e:  # reported below, on the main thread
            errors.append(repr(e))

    print("[gpu-conc] two threads, two streams, one context", flush=True)
    threads = [threading.Thread(target=work, args=(i,)) for i in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    ctx.close()
    assert not errors, errors
    bvh = oracle.bvh_build(tris)
    ob, delta = oracle.default_bounds(tris)
    masks = oracle.object_masks(tris, bvh, 6, delta)
    ora2 = oracle.trace(tris, bvh, rays, mode="raw", R=6, masks=masks, origin_bound=ob)
    ora4 = oracle.trace4(tris, bvh, oracle.bvh4_collapse(bvh), rays, mode="raw", R=6, masks=masks, origin_bound=ob)
    assert all(_same(d, ora2) for d in results[0])
    assert all(_same(d, ora4) for d in results[1])


@pytest.mark.timeout(300)
def test_trace_on_a_side_stream_from_host_rays():
    """Scene build and traces on a stream that is not the current one, with host triangles and rays
    (the binding copies them): the copies are ordered before the library's work on that stream, and
    the results equal the oracle's and those of the current stream."""
    import torch
    assert torch.cuda.is_available()
    from paper_2305_08343_amd import binding, scenes
    tris = scenes.scene_small(0)
    rays = scenes.rays_small(128)
    ctx = binding.Context(0)
    side = torch.cuda.Stream()
    print("[gpu-conc] side stream, host inputs", flush=True)
    sc = binding.Scene(ctx, tris, R=6, mode="raw", width=4, stream=side)
    outs = [sc.trace(rays, stream=side) for _ in range(3)]
    order = sc.ray_order(rays, stream=side)
    side.synchronize()
    base = sc.trace(rays).numpy()
    got = [o.numpy() for o in outs]
    ordr = order.cpu().numpy()
    sc.close()
    ctx.close()
    bvh = oracle.bvh_build(tris)
    ob, delta = oracle.default_bounds(tris)
    masks = oracle.object_masks(tris, bvh, 6, delta)
    ora4 = oracle.trace4(tris, bvh, oracle.bvh4_collapse(bvh), rays, mode="raw", R=6, masks=masks, origin_bound=ob)
    assert _same(base, ora4) and all(_same(d, ora4) for d in got)
    assert sorted(ordr.tolist()) == list(range(rays.shape[0]))


@pytest.mark.timeout(300)
def test_two_threads_build_compressed_scenes_at_once():
    """Two LUT scenes (device codebook selection, Alg. 3, 2-D bit table) built at the same time
    from two host threads on their own streams: codebooks, indices and traces equal the oracle's."""
    import torch
    assert torch.cuda.is_available()
    from paper_2305_08343_amd import binding, scenes
    tris = scenes.scene_small(0)
    rays = scenes.rays_small(96)
    ctx = binding.Context(0)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    cfg = [dict(R=6, K=256, width=4, bit_table=True), dict(R=4, K=128, width=2, bit_table=False)]
    results, errors = [None, None], []

    def work(i):
        try:
            with torch.cuda.stream(streams[i]):
                sc = binding.Scene(ctx, tris, mode="lut", stream=streams[i], **cfg[i])
                exp = sc.export()
                out = sc.trace(torch.from_numpy(rays).cuda(), stream=streams[i])
                streams[i].synchronize()
                results[i] = (exp["codebook"], exp["cidx"], out.numpy())
                sc.close()
        except Exception as e:  # reported below, on the main thread
            errors.append(repr(e))

    print("[gpu-conc] two threads building LUT scenes", flush=True)
    threads = [threading.Thread(target=work, args=(i,)) for i in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    ctx.close()
    assert not errors, errors
    bvh = oracle.bvh_build(tris)
    ob, delta = oracle.default_bounds(tris)
    b4 = oracle.bvh4_collapse(bvh)
    for i, c in enumerate(cfg):
        masks = oracle.object_masks(tris, bvh, c["R"], delta)
        cb, idx = oracle.compress(masks, bvh.slot_boxes(), c["R"], c["K"])
        got_cb, got_idx, dev = results[i]
        assert (got_cb == cb).all() and (got_idx == idx).all()
        kw = dict(mode="lut", R=c["R"], codebook=cb, cidx=idx, origin_bound=ob)
        ora = oracle.trace4(tris, bvh, b4, rays, **kw) if c["width"] == 4 else oracle.trace(tris, bvh, rays, **kw)
        assert _same(dev, ora)
