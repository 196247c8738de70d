"""sc_trace_noalloc (the allocation-free trace: queue counters and sort
workspace in the library's fixed per-GPU scratch array) against sc_trace, the
entry point it mirrors, through the C ABI: two calls in a row, the second on
fewer rays, unsorted and sorted, binary and 4-wide scenes, raw and compressed
masks; results bit-exact (and equal to the oracle on the small scene). Also
the size limit of a sorted call."""
import ctypes as C

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def _call(lib, fn, scene, rays, n, flags, hits, extra, stream):
    return getattr(lib, fn)(scene.handle, C.c_void_p(rays.data_ptr()), n, flags, C.c_void_p(hits.data_ptr()),
                            C.c_void_p(extra.data_ptr()), None, C.c_void_p(stream.cuda_stream))


def _host(hits, extra, n):
    h = hits[:n].cpu().numpy().view(np.uint32)
    e = extra[:n].cpu().numpy().view(np.uint32)
    return np.concatenate([h, e], axis=1)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("width,mode,R", [(2, "raw", 6), (4, "raw", 6), (4, "lut", 6), (4, "none", 6),
                                          (4, "raw", 4)])
def test_noalloc_equals_trace_two_calls_second_smaller(width, mode, R):
    import torch
    from paper_2305_08343_amd import binding, scenes
    assert torch.cuda.is_available()
    lib = binding.load()
    tris = scenes.scene_small(0)
    rays_np = scenes.rays_small(256)
    aimed = scenes.random_rays(20000, 3)
    rays_np = np.concatenate([rays_np, aimed])
    ctx = binding.Context(0)
    stream = torch.cuda.current_stream()
    print(f"[no-alloc] width {width} mode {mode} R {R}", flush=True)
    scene = binding.Scene(ctx, tris, R=R, mode=mode, width=width, K=256)
    rays = torch.from_numpy(rays_np).cuda()
    n1 = rays.shape[0]
    n2 = 4099  # a smaller second call with a ragged last wave
    for sort in (0, 1):
        for cull in (True, False):
            flags = (binding.SC_TRACE_CULL if cull else 0) | (binding.SC_TRACE_SORT if sort else 0)
            ref_h = torch.empty((n1, 4), dtype=torch.int32, device="cuda")
            ref_e = torch.empty((n1, 2), dtype=torch.int32, device="cuda")
            assert _call(lib, "sc_trace", scene, rays, n1, flags, ref_h, ref_e, stream) == 0
            ref = _host(ref_h, ref_e, n1)
            hits = torch.full((n1, 4), -7, dtype=torch.int32, device="cuda")
            extra = torch.full((n1, 2), -7, dtype=torch.int32, device="cuda")
            assert _call(lib, "sc_trace_noalloc", scene, rays, n1, flags, hits, extra, stream) == 0, \
                lib.sc_last_error()
            got1 = _host(hits, extra, n1)
            hits.fill_(-7)
            extra.fill_(-7)
            # the second call: the last n2 rays (another ray range, fewer rays)
            sub = rays[n1 - n2:].contiguous()
            assert _call(lib, "sc_trace_noalloc", scene, sub, n2, flags, hits, extra, stream) == 0, \
                lib.sc_last_error()
            got2 = _host(hits, extra, n2)
            rest = hits[n2:].cpu().numpy()
            torch.cuda.synchronize()
            assert (got1 == ref).all(), (sort, cull)
            assert (got2 == ref[n1 - n2:]).all(), (sort, cull)
            assert (rest == -7).all()  # nothing written beyond the second call's rays
            if sort == 0 and cull:
                culled = ref
    if mode == "raw" and width == 2 and R == 6:
        ref = culled
        bvh = oracle.bvh_build(tris)
        ob, delta = oracle.default_bounds(tris)
        ora = oracle.trace(tris, bvh, rays_np, mode="raw", R=6, masks=oracle.object_masks(tris, bvh, 6, delta),
                           origin_bound=ob)
        assert (ref[:, 0] == ora.prim).all() and (ref[:, 1] == ora.t.view(np.uint32)).all()
        assert (ref[:, 2] == ora.box_tests).all() and (ref[:, 3] == ora.tri_tests).all()
        assert (ref[:, 4] == ora.mask_tests).all() and (ref[:, 5] == ora.mask_culls).all()
    scene.close()
    ctx.close()


@pytest.mark.timeout(300)
def test_noalloc_sorted_size_limit_and_launch_shape_sort():
    """A sorted call above the scratch's 4,194,304 rays is refused before any HIP call (the rays
    pointer is never read); an unsorted call of the same size runs; the context's launch shape
    can ask for the sort too."""
    import torch
    from paper_2305_08343_amd import binding, scenes
    lib = binding.load()
    tris = scenes.scene_small(0)
    ctx = binding.Context(0)
    scene = binding.Scene(ctx, tris, R=6, mode="raw", width=4)
    stream = torch.cuda.current_stream()
    big = (1 << 22) + 1
    rays = torch.from_numpy(np.tile(scenes.rays_small(64), (big // 4096 + 1, 1))[:big]).cuda()
    hits = torch.empty((big, 4), dtype=torch.int32, device="cuda")
    extra = torch.empty((big, 2), dtype=torch.int32, device="cuda")
    print("[no-alloc] size limit", flush=True)
    assert _call(lib, "sc_trace_noalloc", scene, rays, big, binding.SC_TRACE_SORT | binding.SC_TRACE_CULL,
                 hits, extra, stream) == 1
    assert b"4194304" in lib.sc_last_error()
    assert _call(lib, "sc_trace_noalloc", scene, rays, big, binding.SC_TRACE_CULL, hits, extra, stream) == 0
    ref_h = torch.empty_like(hits)
    ref_e = torch.empty_like(extra)
    assert _call(lib, "sc_trace", scene, rays, big, binding.SC_TRACE_CULL, ref_h, ref_e, stream) == 0
    torch.cuda.synchronize()
    assert torch.equal(hits, ref_h) and torch.equal(extra, ref_e)
    # a launch shape with sorting on: the same refusal above the limit, and equal results below it
    t = ctx.get_tune()
    ctx.set_tune(t["block"], t["stack"], t["chunk"], t["parts"], t["waves"], 1, t["codebook"], t["gather"],
                 t["refill"])
    assert _call(lib, "sc_trace_noalloc", scene, rays, big, binding.SC_TRACE_CULL, hits, extra, stream) == 1
    n = 1 << 22
    assert _call(lib, "sc_trace_noalloc", scene, rays, n, binding.SC_TRACE_CULL, hits, extra, stream) == 0
    torch.cuda.synchronize()
    assert torch.equal(hits[:n], ref_h[:n]) and torch.equal(extra[:n], ref_e[:n])
    scene.close()
    ctx.close()
