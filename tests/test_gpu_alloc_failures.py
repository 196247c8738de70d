"""Allocation failures forced from the host: a device allocator that refuses its k-th request.

Every refusal surfaces as SC_ERR_OOM from the call that needed the memory, before any kernel
uses the missing buffer; the failed call leaves nothing allocated beyond what the context itself
keeps (its ray-queue counters and ray-mask tables); the context after a failed build and the
scene after a failed trace stay usable, with the results of an undisturbed run; and destroying
everything returns every allocation. The refusal is a host decision, so every kernel that runs
exits normally."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SC_ERR_OOM = 3


class Refusing:
    """Device memory from torch's caching allocator, refusing request number `refuse_at` (1-based;
    0 = never); records the live allocations and any free of an unknown pointer."""

    def __init__(self, device=0):
        self.device = device
        self.calls = 0
        self.refuse_at = 0
        self.live = {}
        self.errors = []

    def alloc(self, nbytes, stream):
        import torch
        self.calls += 1
        if self.calls == self.refuse_at:
            return 0
        p = torch.cuda.caching_allocator_alloc(nbytes, self.device, stream)
        self.live[p] = nbytes
        return p

    def free(self, ptr, nbytes, stream):
        import torch
        if self.live.pop(ptr, None) != nbytes:
            self.errors.append((ptr, nbytes))
        torch.cuda.caching_allocator_delete(ptr)

    def sizes(self):
        return sorted(self.live.values())


BUILDS = {
    "lut6w4b": dict(R=6, mode="lut", K=256, width=4, bit_table=True),
    "raw6w4": dict(R=6, mode="raw", width=4),
    "raw4_approx3": dict(R=4, mode="raw", approx_levels=3),
    "sparse6": dict(R=6, mode="sparse"),
    "none4q": dict(R=6, mode="none", width=4, quantise=True),
}


def _build(ctx, tris, name, placement=None):
    from paper_2305_08343_amd import binding
    kw = dict(BUILDS[name])
    if name == "sparse6":
        kw["placement"] = placement
    return binding.Scene(ctx, tris, **kw)


def _same(a, b):
    return all((a[k] == b[k]).all() for k in ("prim", "box_tests", "tri_tests", "mask_tests", "mask_culls")) and \
        (a["t"].view(np.uint32) == b["t"].view(np.uint32)).all()


@pytest.mark.parametrize("name", list(BUILDS))
def test_refused_allocations_in_context_build_and_trace(small_scene, small_oracle, name):
    from paper_2305_08343_amd import binding
    tris, rays = small_scene
    S = 2 * small_oracle["bvh"].n_inner
    placement = (np.random.default_rng(3).random(S) < 0.3).astype(np.uint8)
    build = lambda c: _build(c, tris, name, placement)  # noqa: E731
    # an undisturbed run: how many requests the context and the build make, and what the context keeps
    A = Refusing()
    ctx = binding.Context(0, allocator=(A.alloc, A.free))
    n_ctx = A.calls
    s = build(ctx)
    n_build = A.calls - n_ctx
    ref = s.trace(rays).numpy()
    s.close()
    kept = A.sizes()
    ctx.close()
    assert not A.live and not A.errors
    assert n_build >= 3
    print(f"[gpu-alloc] {name}: context {n_ctx} requests, build {n_build}", flush=True)

    for k in range(1, n_ctx + n_build + 1):
        print(f"[gpu-alloc] {name}: refusing request {k}", flush=True)
        A = Refusing()
        A.refuse_at = k
        if k <= n_ctx:
            with pytest.raises(binding.SubcullError) as ei:
                binding.Context(0, allocator=(A.alloc, A.free))
            assert ei.value.status == SC_ERR_OOM
            assert not A.live and not A.errors
            continue
        ctx = binding.Context(0, allocator=(A.alloc, A.free))
        with pytest.raises(binding.SubcullError) as ei:
            build(ctx)
        assert ei.value.status == SC_ERR_OOM, ei.value
        # nothing of the failed scene is left: the live sizes are a part of what the context keeps
        rest = list(kept)
        for b in A.sizes():
            assert b in rest, (k, b, kept)
            rest.remove(b)
        # the context still builds, and the scene traces as in the undisturbed run
        s = build(ctx)
        assert _same(s.trace(rays).numpy(), ref)
        s.close()
        ctx.close()
        assert not A.live and not A.errors

    # a trace whose ray-order workspace is refused fails alone: the scene keeps working
    A = Refusing()
    ctx = binding.Context(0, allocator=(A.alloc, A.free))
    s = build(ctx)
    A.refuse_at = A.calls + 1
    with pytest.raises(binding.SubcullError) as ei:
        s.trace(rays, sort=True)
    assert ei.value.status == SC_ERR_OOM
    assert _same(s.trace(rays, sort=True).numpy(), ref)
    assert _same(s.trace(rays).numpy(), ref)
    s.close()
    ctx.close()
    assert not A.live and not A.errors


@pytest.mark.parametrize("graph", [True, False])
def test_refused_allocations_in_batched_traces(small_scene, graph):
    """A sorted batch of two scenes: each request of sc_batch_create (descriptors, counters,
    ray-order workspace) or of sc_trace_batch (descriptors, workspace) refused in turn."""
    from paper_2305_08343_amd import binding, scenes
    tris, rays = small_scene
    tris2 = scenes.micro_scene(5, 64)
    rays2 = np.concatenate([rays[:5000], scenes.random_rays(333, 9)])
    A = Refusing()
    ctx = binding.Context(0, allocator=(A.alloc, A.free))
    s1 = binding.Scene(ctx, tris, R=4, mode="raw", width=4)
    s2 = binding.Scene(ctx, tris2, R=4, mode="raw", width=4)
    want = [s1.trace(rays).numpy(), s2.trace(rays2).numpy()]
    start = A.calls
    b = binding.Batch(ctx, [(s1, rays), (s2, rays2)], graph=graph, sort=True)
    if not graph:
        b.launch()
    n_req = A.calls - start
    b.close()
    assert n_req >= 2
    print(f"[gpu-alloc] batch graph={graph}: {n_req} requests", flush=True)
    for k in range(1, n_req + 1):
        print(f"[gpu-alloc] batch graph={graph}: refusing request {k}", flush=True)
        A.refuse_at = A.calls + k
        held = A.sizes()
        with pytest.raises(binding.SubcullError) as ei:
            b = binding.Batch(ctx, [(s1, rays), (s2, rays2)], graph=graph, sort=True)
            b.launch()
        assert ei.value.status == SC_ERR_OOM, ei.value
        b = None
        assert A.sizes() == held
        A.refuse_at = 0
        b = binding.Batch(ctx, [(s1, rays), (s2, rays2)], graph=graph, sort=True)
        b.launch()
        import torch
        torch.cuda.synchronize()
        assert _same(b.results(0).numpy(), want[0]) and _same(b.results(1).numpy(), want[1])
        b.close()
    s1.close()
    s2.close()
    ctx.close()
    assert not A.live and not A.errors
