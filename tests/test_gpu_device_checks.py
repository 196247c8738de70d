"""The traversal kernels with device checks (sc_set_device_checks): on valid
scenes they change nothing -- hits and every count equal the unchecked
kernels', in every node width, mask mode and child-box storage, through
sc_trace, sc_trace_noalloc and batches (direct and graph) -- and no check
fails; the same checked trace run twice is identical. Each check is then made
to fail by lowering its limit below the scene's own (sc_set_check_limits):
the buffers keep their size, so the failing check guards no access out of
range; the launch completes, the check's bit is set, and restoring the
limits restores the unchecked results."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

FIELDS = ("prim", "t", "box_tests", "tri_tests", "mask_tests", "mask_culls")

CONFIGS = [
    dict(width=2, mode="none", R=6),
    dict(width=2, mode="raw", R=6),
    dict(width=2, mode="raw", R=4),
    dict(width=2, mode="lut", R=6, K=256),
    dict(width=2, mode="lut", R=6, K=4096, bit_table=True),
    dict(width=4, mode="none", R=6),
    dict(width=4, mode="raw", R=4),
    dict(width=4, mode="raw", R=6),
    dict(width=4, mode="lut", R=6, K=4096),
    dict(width=4, mode="lut", R=6, K=4096, bit_table=True),
    dict(width=4, mode="raw", R=4, quantise=True),
    dict(width=4, mode="none", R=6, quantise=True),
]


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_2305_08343_amd import binding
    c = binding.Context(0, checks=False)
    yield c
    c.close()


@pytest.fixture(scope="module")
def rays(small_scene):
    import torch
    from paper_2305_08343_amd import scenes
    _, r = small_scene
    return torch.from_numpy(np.concatenate([r, scenes.random_rays(20000, 5)])).cuda()


def _same(a, b, what):
    for f in FIELDS:
        x, y = a[f], b[f]
        if f == "t":
            x, y = x.view(np.uint32), y.view(np.uint32)
        assert (x == y).all(), f"{what}: {f} differs on {(x != y).sum()} rays"


def _name(cfg):
    return "-".join(f"{k}{v}" for k, v in cfg.items())


@pytest.mark.timeout(300)
@pytest.mark.parametrize("cfg", CONFIGS, ids=_name)
def test_checked_kernels_change_nothing(ctx, small_scene, rays, cfg):
    import torch
    from paper_2305_08343_amd import binding
    tris, _ = small_scene
    print(f"[gpu-checks] {_name(cfg)}", flush=True)
    s = binding.Scene(ctx, tris, **cfg)
    ctx.set_device_checks(False)
    ref = s.trace(rays).numpy()
    ctx.set_device_checks(True)
    assert ctx.check_flags(reset=True) == 0
    got = s.trace(rays).numpy()
    again = s.trace(rays).numpy()
    flags = ctx.check_flags(reset=True)
    ctx.set_device_checks(False)
    s.close()
    _same(got, ref, "checked vs unchecked")
    _same(again, got, "checked, run twice")
    assert flags == 0, f"a check failed on a valid scene: bits {flags:#x}"


@pytest.mark.timeout(300)
def test_checked_noalloc_and_batches(ctx, small_scene, rays):
    import torch
    from paper_2305_08343_amd import binding
    tris, _ = small_scene
    lib = binding.load()
    s = binding.Scene(ctx, tris, R=4, mode="raw", width=4, quantise=True)
    s2 = binding.Scene(ctx, tris[: tris.shape[0] // 2], R=4, mode="raw", width=4, quantise=True)
    half = rays[:30000]
    ctx.set_device_checks(False)
    ref = [s.trace(rays).numpy(), s2.trace(half).numpy()]
    ctx.set_device_checks(True)
    ctx.check_flags(reset=True)
    # the allocation-free entry point runs the same checked instances
    n = rays.shape[0]
    hits = torch.empty((n, 4), dtype=torch.int32, device="cuda")
    extra = torch.empty((n, 2), dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    print("[gpu-checks] noalloc", flush=True)
    assert lib.sc_trace_noalloc(s.handle, C.c_void_p(rays.data_ptr()), n, binding.SC_TRACE_CULL,
                                C.c_void_p(hits.data_ptr()), C.c_void_p(extra.data_ptr()), None,
                                C.c_void_p(stream.cuda_stream)) == 0, lib.sc_last_error()
    _same(binding.TraceResult(hits, extra).numpy(), ref[0], "checked noalloc")
    for graph in (False, True):
        print(f"[gpu-checks] batch graph={graph}", flush=True)
        b = binding.Batch(ctx, [(s, rays), (s2, half)], graph=graph)
        b.launch()
        torch.cuda.synchronize()
        _same(b.results(0).numpy(), ref[0], f"checked batch item 0, graph={graph}")
        _same(b.results(1).numpy(), ref[1], f"checked batch item 1, graph={graph}")
        b.close()
    assert ctx.check_flags(reset=True) == 0
    ctx.set_device_checks(False)
    s.close()
    s2.close()


@pytest.mark.timeout(300)
@pytest.mark.parametrize("width", [2, 4])
def test_lowered_limits_make_each_check_fail(ctx, small_scene, rays, width):
    from paper_2305_08343_amd import binding
    tris, _ = small_scene
    s = binding.Scene(ctx, tris, R=6, mode="raw", width=width)
    ctx.set_device_checks(False)
    ref = s.trace(rays).numpy()
    ctx.set_device_checks(True)
    ctx.check_flags(reset=True)
    for limits, bit in (((1, 0, 0), binding.SC_CHECK_STACK), ((0, 1, 0), binding.SC_CHECK_NODE),
                        ((0, 0, 1), binding.SC_CHECK_TRI)):
        print(f"[gpu-checks] width {width} limits {limits}", flush=True)
        ctx.set_check_limits(*limits)
        got = s.trace(rays).numpy()
        flags = ctx.check_flags(reset=True)
        assert flags == bit, f"limits {limits}: bits {flags:#x}, expected {bit:#x}"
        # a failed check ends rays or drops stack entries: never a hit the unchecked trace lacks
        found = got["prim"] != 0xFFFFFFFF
        assert (ref["prim"][found] != 0xFFFFFFFF).all()
        assert (got["t"][found] >= ref["t"][found]).all()
    ctx.set_check_limits(0, 0, 0)
    _same(s.trace(rays).numpy(), ref, "limits restored")
    assert ctx.check_flags(reset=True) == 0
    ctx.set_device_checks(False)
    s.close()
