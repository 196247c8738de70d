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
