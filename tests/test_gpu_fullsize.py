"""GPU parity at the full workload sizes, in the launch configuration bench.py times.

hair_1m (1,000,002 tris, 4,147,200 rays): BVH, masks (R = 4, 6), codebook and
indices, and every ray's hit/t/counts in the plain, raw R = 6, raw R = 4 and
compressed modes, all bit-exact against the oracle; the 4-wide modes the benchmark
times (216-bit masks with exact and quantised child boxes, plain quantised) on
every ray in their stored launch shapes.

curly_12m (12,000,000 tris, 8,000,000 rays): BVH bit-exact; masks of a slot
sample; every 64th ray bit-exact in every mode (oracle with all masks); and on
all 8M rays the properties that hold at any size: culled hits equal unculled
hits, per-ray counts none >= compressed >= raw, every stored codebook entry
contains its slot's exact mask. The 4-wide modes bench.py times on this
workload (216-bit masks compressed to 4,096 codebook entries on exact and on
quantised child boxes, tested through the 2-D bit table or by codebook fetch,
64-bit raw masks on every slot and on leaf slots, plain traversal), each
traced in the launch shape bench.py stores for it: 4-wide nodes, codebook,
indices and bit table bit-exact against the oracle, every 64th ray
bit-exact against the oracle's 4-wide traversal, and on all 8M rays hits equal
to the unculled ones with counts none >= compressed and none >= leaf-slot >=
every-slot raw masks.
"""
import numpy as np
import pytest

import oracle
from paper_2305_08343_amd import scenes

pytestmark = pytest.mark.gpu


def _say(request, msg):
    capman = request.config.pluginmanager.getplugin("capturemanager")
    with capman.global_and_fixture_disabled():
        print(f"[gpu-full] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_2305_08343_amd import binding
    c = binding.Context(0)  # default launch shape, as in bench.py
    yield c
    c.close()


def _compare(dev, ora, sel=None):
    sel = slice(None) if sel is None else sel
    for k, o in (("prim", ora.prim), ("box_tests", ora.box_tests), ("tri_tests", ora.tri_tests),
                 ("mask_tests", ora.mask_tests), ("mask_culls", ora.mask_culls)):
        d = dev[k][sel]
        bad = np.flatnonzero(d != o)
        assert bad.size == 0, f"{k}: {bad.size} rays differ, first {bad[:5]}"
    assert (dev["t"][sel].view(np.uint32) == ora.t.view(np.uint32)).all()


def _superset(big, small):
    return ((small & ~big) == 0).all(axis=-1)


# --------------------------------------------------------------------- hair_1m
@pytest.fixture(scope="module")
def hair(request):
    _say(request, "hair_1m: generating scene and rays")
    tris = scenes.scene_hair_1m(1)
    rays = scenes.rays_hair_1m(tris, 1)
    nt = oracle.cpu_threads()
    _say(request, f"hair_1m: oracle BVH + masks on {nt} threads")
    bvh = oracle.bvh_build(tris)
    ob, delta = oracle.default_bounds(tris)
    return {"tris": tris, "rays": rays, "bvh": bvh, "ob": ob, "delta": delta, "nt": nt,
            "masks4": oracle.object_masks(tris, bvh, 4, delta, nthreads=nt),
            "masks6": oracle.object_masks(tris, bvh, 6, delta, nthreads=nt)}


@pytest.mark.timeout(600)
def test_hair_1m_all_rays_bit_exact(request, ctx, hair):
    from paper_2305_08343_amd import binding
    tris, rays, bvh = hair["tris"], hair["rays"], hair["bvh"]
    for mode, R in (("none", 6), ("raw", 6), ("raw", 4)):
        _say(request, f"hair_1m mode={mode} R={R}: build, export, trace {rays.shape[0]} rays")
        s = binding.Scene(ctx, tris, R=R, mode=mode)
        exp = s.export()
        assert (exp["cbox"].view(np.uint32) == bvh.cbox.view(np.uint32)).all()
        assert (exp["cref"] == bvh.cref).all() and (exp["perm"] == bvh.perm).all()
        kw = dict(origin_bound=hair["ob"], nthreads=hair["nt"])
        if mode == "raw":
            assert (exp["masks"] == hair[f"masks{R}"]).all()
            kw.update(mode="raw", R=R, masks=hair[f"masks{R}"])
        dev = s.trace(rays).numpy()
        s.close()
        _compare(dev, oracle.trace(tris, bvh, rays, **kw))


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name", ["raw6w4q", "raw6w4", "nonew4q"])
def test_hair_1m_4_wide_all_rays_bit_exact_in_bench_launch_shape(request, ctx, hair, name):
    """The benchmark's 4-wide modes (216-bit masks with quantised and with exact child boxes,
    and the plain quantised traversal) on every ray, in the launch shape bench.py stores for them."""
    import bench
    from paper_2305_08343_amd import binding
    tris, rays, bvh = hair["tris"], hair["rays"], hair["bvh"]
    spec = bench.MODES[name]
    q = spec.get("quantise", False)
    _say(request, f"hair_1m {name}: build, export, trace {rays.shape[0]} rays in shape {spec['tune']}")
    b4 = oracle.bvh4_collapse(bvh)
    if q:
        b4 = oracle.decoded_bvh4(b4, oracle.quantise4(b4))
        bq = oracle.with_slot_boxes(bvh, b4)
    else:
        bq = bvh
    kw = dict(origin_bound=hair["ob"], nthreads=hair["nt"])
    s = binding.Scene(ctx, tris, R=spec["R"], mode=spec["mode"], width=4, quantise=q)
    e4 = s.export4()
    assert (e4["box4"].view(np.uint32) == b4.box4.view(np.uint32)).all() and (e4["ref4"] == b4.ref4).all()
    if spec["mode"] == "raw":
        masks = hair["masks6"] if not q else oracle.object_masks(tris, bq, 6, hair["delta"], nthreads=hair["nt"])
        assert (s.export()["masks"] == masks).all()
        kw.update(mode="raw", R=6, masks=masks)
    try:
        ctx.set_tune(*spec["tune"])
        dev = s.trace(rays).numpy()
    finally:
        ctx.set_tune()
        s.close()
    _compare(dev, oracle.trace4(tris, bq, b4, rays, **kw))


@pytest.mark.timeout(600)
def test_hair_1m_compressed_bit_exact(request, ctx, hair):
    from paper_2305_08343_amd import binding
    tris, rays, bvh = hair["tris"], hair["rays"], hair["bvh"]
    _say(request, "hair_1m compressed K=4096: codebook, indices, every 2nd ray")
    s = binding.Scene(ctx, tris, R=6, mode="lut", K=4096)
    exp = s.export()
    cb, idx = oracle.compress(hair["masks6"], bvh.slot_boxes(), 6, 4096)
    assert (exp["codebook"] == cb).all() and (exp["cidx"] == idx).all()
    sel = rays[::2]
    dev = s.trace(sel).numpy()
    s.close()
    _compare(dev, oracle.trace(tris, bvh, sel, mode="lut", R=6, codebook=cb, cidx=idx,
                               origin_bound=hair["ob"], nthreads=hair["nt"]))


@pytest.mark.timeout(600)
@pytest.mark.parametrize("K", [64, 256])
def test_hair_1m_compressed_r4_codebook_bit_exact(request, ctx, hair, K):
    """64-bit masks (one word a mask: the device value sort in 2 rounds) compressed to small codebooks
    over the 1M-triangle scene's 602,340 slots: codebook, indices and every 4th ray."""
    from paper_2305_08343_amd import binding
    tris, rays, bvh = hair["tris"], hair["rays"], hair["bvh"]
    _say(request, f"hair_1m compressed R=4 K={K}: codebook, indices, every 4th ray")
    s = binding.Scene(ctx, tris, R=4, mode="lut", K=K)
    exp = s.export()
    cb, idx = oracle.compress(hair["masks4"], bvh.slot_boxes(), 4, K)
    assert (exp["codebook"] == cb).all() and (exp["cidx"] == idx).all()
    sel = rays[::4]
    dev = s.trace(sel).numpy()
    s.close()
    _compare(dev, oracle.trace(tris, bvh, sel, mode="lut", R=4, codebook=cb, cidx=idx,
                               origin_bound=hair["ob"], nthreads=hair["nt"]))


# ------------------------------------------------------------------- curly_12m
@pytest.fixture(scope="module")
def curly(request):
    _say(request, "curly_12m: generating 12M tris, 8M rays")
    tris = scenes.scene_curly_12m(2)
    rays = scenes.rays_curly_12m(tris)
    nt = oracle.cpu_threads()
    _say(request, f"curly_12m: oracle BVH on {nt} threads")
    bvh = oracle.bvh_build(tris)
    ob, delta = oracle.default_bounds(tris)
    return {"tris": tris, "rays": rays, "bvh": bvh, "ob": ob, "delta": delta, "nt": nt}


@pytest.fixture(scope="module")
def curly_dev(request, ctx, curly):
    """Device results for all 8M rays in the three modes, plus exports."""
    from paper_2305_08343_amd import binding
    out = {}
    for mode, R in (("none", 6), ("lut", 6), ("raw", 6)):
        _say(request, f"curly_12m mode={mode}: device build + trace of 8M rays")
        s = binding.Scene(ctx, curly["tris"], R=R, mode=mode, K=4096)
        out[mode] = s.trace(curly["rays"]).numpy()
        if mode != "none":
            e = s.export()
            out[f"export_{mode}"] = {k: e[k] for k in ("masks", "codebook", "cidx")}
        else:
            out["export_none"] = s.export()
        s.close()
    return out


@pytest.mark.timeout(900)
def test_curly_12m_bvh_and_sampled_masks(request, curly, curly_dev):
    bvh = curly["bvh"]
    exp = curly_dev["export_none"]
    _say(request, "curly_12m: BVH export vs oracle")
    assert exp["cbox"].shape == bvh.cbox.shape
    assert (exp["cbox"].view(np.uint32) == bvh.cbox.view(np.uint32)).all()
    assert (exp["cref"] == bvh.cref).all() and (exp["range"] == bvh.range).all()
    assert (exp["perm"] == bvh.perm).all()
    rng = np.random.default_rng(0)
    S = 2 * bvh.n_inner
    slots = np.unique(np.concatenate([rng.integers(0, S, 3000), np.arange(8)]))
    _say(request, f"curly_12m: oracle masks of {slots.size} sampled slots")
    m = oracle.slot_masks(curly["tris"], bvh, slots, 6, curly["delta"], nthreads=curly["nt"])
    assert (curly_dev["export_raw"]["masks"][slots] == m).all()
    assert (curly_dev["export_lut"]["masks"][slots] == m).all()


@pytest.mark.timeout(900)
def test_curly_12m_properties_all_rays(request, curly_dev):
    _say(request, "curly_12m: properties over all 8M rays")
    n, l, r = curly_dev["none"], curly_dev["lut"], curly_dev["raw"]
    for d in (l, r):
        assert (d["prim"] == n["prim"]).all()
        assert (d["t"].view(np.uint32) == n["t"].view(np.uint32)).all()
    for f in ("box_tests", "tri_tests"):
        assert (n[f] >= l[f]).all() and (l[f] >= r[f]).all()
    assert (r["mask_culls"] <= r["mask_tests"]).all()
    e = curly_dev["export_lut"]
    assert _superset(e["codebook"][e["cidx"]], e["masks"]).all()
    pc = np.unpackbits(e["codebook"].view(np.uint8), axis=1).sum(1)
    assert (np.diff(pc) >= 0).all()


@pytest.fixture(scope="module")
def curly_masks(request, curly):
    """Oracle masks of every slot (R = 6) and the K = 4096 codebook with Alg. 3 indices."""
    tris, bvh = curly["tris"], curly["bvh"]
    _say(request, "curly_12m: oracle masks (all slots, R=6) and codebook K=4096 + Alg. 3")
    masks = oracle.object_masks(tris, bvh, 6, curly["delta"], nthreads=curly["nt"])
    cb, idx = oracle.compress(masks, bvh.slot_boxes(), 6, 4096)
    return {"masks6": masks, "cb": cb, "idx": idx}


@pytest.mark.timeout(900)
def test_curly_12m_sampled_rays_bit_exact(request, curly, curly_dev, curly_masks):
    tris, bvh, rays = curly["tris"], curly["bvh"], curly["rays"]
    sel = slice(None, None, 64)
    sample = rays[sel]
    _say(request, f"curly_12m: oracle traces of {sample.shape[0]} sampled rays, plain")
    _compare(curly_dev["none"], oracle.trace(tris, bvh, sample, origin_bound=curly["ob"],
                                             nthreads=curly["nt"]), sel)
    masks = curly_masks["masks6"]
    assert (curly_dev["export_raw"]["masks"] == masks).all()
    _compare(curly_dev["raw"], oracle.trace(tris, bvh, sample, mode="raw", R=6, masks=masks,
                                            origin_bound=curly["ob"], nthreads=curly["nt"]), sel)
    cb, idx = curly_masks["cb"], curly_masks["idx"]
    assert (curly_dev["export_lut"]["codebook"] == cb).all()
    assert (curly_dev["export_lut"]["cidx"] == idx).all()
    _compare(curly_dev["lut"], oracle.trace(tris, bvh, sample, mode="lut", R=6, codebook=cb, cidx=idx,
                                            origin_bound=curly["ob"], nthreads=curly["nt"]), sel)


# 4-wide modes of the curly benchmark, each in the launch shape bench.py stores for it there
CURLY4 = ["lut6w4b", "lut6w4", "lut6w4q", "raw4w4", "raw4w4l", "nonew4", "nonew4q"]


@pytest.fixture(scope="module")
def curly4_dev(request, ctx, curly):
    import bench
    from paper_2305_08343_amd import binding
    out = {}
    for name in CURLY4:
        spec = bench.MODES[name]
        shape = bench.stored_tune(name, "curly_12m")
        _say(request, f"curly_12m {name}: device build + trace of 8M rays in shape {shape}")
        s = binding.Scene(ctx, curly["tris"], R=spec["R"], mode=spec["mode"], K=spec.get("K", 4096), width=4,
                          quantise=spec.get("quantise", False), mask_slots=spec.get("mask_slots", "all"),
                          bit_table=spec.get("bit_table", False))
        try:
            ctx.set_tune(*shape)
            out[name] = s.trace(curly["rays"]).numpy()
        finally:
            ctx.set_tune()
        out[f"{name}/export4"] = s.export4()
        if spec["mode"] == "lut":
            e = s.export()
            out[f"{name}/cb"] = (e["codebook"], e["cidx"])
        if spec.get("bit_table"):
            out[f"{name}/bits"] = s.export_bit_table()
        s.close()
    return out


@pytest.fixture(scope="module")
def curly4_oracle(request, curly, curly_masks):
    """The oracle's 4-wide BVH (exact and decoded quantised boxes) and the masks / codebooks on
    the slot boxes each mode's traversal tests."""
    tris, bvh, delta, nt = curly["tris"], curly["bvh"], curly["delta"], curly["nt"]
    b4 = oracle.bvh4_collapse(bvh)
    d4 = oracle.decoded_bvh4(b4, oracle.quantise4(b4))
    bq = oracle.with_slot_boxes(bvh, d4)
    _say(request, "curly_12m: oracle masks R=4 (exact boxes), R=6 and codebook on the decoded boxes")
    masks4 = oracle.object_masks(tris, bvh, 4, delta, nthreads=nt)
    masks6q = oracle.object_masks(tris, bq, 6, delta, nthreads=nt)
    cbq, idxq = oracle.compress(masks6q, bq.slot_boxes(), 6, 4096)
    return {"b4": b4, "d4": d4, "bq": bq,
            "lut6w4": (bvh, b4, dict(mode="lut", R=6, codebook=curly_masks["cb"], cidx=curly_masks["idx"])),
            # the bit table answers the same test as codebook fetch + AND
            "lut6w4b": (bvh, b4, dict(mode="lut", R=6, codebook=curly_masks["cb"], cidx=curly_masks["idx"])),
            "lut6w4q": (bq, d4, dict(mode="lut", R=6, codebook=cbq, cidx=idxq)),
            "raw4w4": (bvh, b4, dict(mode="raw", R=4, masks=masks4)),
            "raw4w4l": (bvh, b4, dict(mode="raw", R=4, masks=oracle.leaf_slot_masks(masks4, bvh, 4))),
            "nonew4": (bvh, b4, {}),
            "nonew4q": (bq, d4, {})}


@pytest.mark.timeout(900)
def test_curly_12m_4_wide_nodes_and_codebooks(request, curly4_dev, curly4_oracle, curly_masks):
    _say(request, "curly_12m: 4-wide nodes, codebooks and indices vs oracle")
    for name in CURLY4:
        q = name.endswith("q")
        ob4 = curly4_oracle["d4" if q else "b4"]
        e4 = curly4_dev[f"{name}/export4"]
        assert (e4["box4"].view(np.uint32) == ob4.box4.view(np.uint32)).all(), name
        assert (e4["ref4"] == ob4.ref4).all() and (e4["src4"] == ob4.src4).all(), name
    for name in ("lut6w4b", "lut6w4", "lut6w4q"):
        cb, idx = curly4_dev[f"{name}/cb"]
        want = curly4_oracle[name][2]
        assert (cb == want["codebook"]).all() and (idx == want["cidx"]).all(), name
    _say(request, "curly_12m: 2-D bit table (R^6 x 4096 bits) vs oracle")
    assert (curly4_dev["lut6w4b/bits"] == oracle.bit_table(6, curly_masks["cb"])).all()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name", CURLY4)
def test_curly_12m_4_wide_sampled_rays_bit_exact(request, curly, curly4_dev, curly4_oracle, name):
    sel = slice(None, None, 64)
    sample = curly["rays"][sel]
    bvh, b4, kw = curly4_oracle[name]
    _say(request, f"curly_12m {name}: oracle 4-wide trace of {sample.shape[0]} sampled rays")
    ora = oracle.trace4(curly["tris"], bvh, b4, sample, origin_bound=curly["ob"], nthreads=curly["nt"], **kw)
    _compare(curly4_dev[name], ora, sel)


@pytest.mark.timeout(900)
def test_curly_12m_4_wide_properties_all_rays(request, curly_dev, curly4_dev):
    _say(request, "curly_12m: 4-wide properties over all 8M rays")
    plain = curly4_dev["nonew4"]
    for name in CURLY4:
        d = curly4_dev[name]
        assert (d["prim"] == plain["prim"]).all(), name
        assert (d["t"].view(np.uint32) == plain["t"].view(np.uint32)).all(), name
        assert (d["mask_culls"] <= d["mask_tests"]).all(), name
    # and the binary BVH's hits
    assert (curly_dev["none"]["prim"] == plain["prim"]).all()
    assert (curly_dev["none"]["t"].view(np.uint32) == plain["t"].view(np.uint32)).all()
    for f in ("box_tests", "tri_tests"):
        # same tree: culling only removes tests; leaf-slot masks are a superset of all-slot masks
        assert (plain[f] >= curly4_dev["lut6w4"][f]).all(), f
        assert (plain[f] >= curly4_dev["raw4w4l"][f]).all(), f
        assert (curly4_dev["raw4w4l"][f] >= curly4_dev["raw4w4"][f]).all(), f
        assert (curly4_dev["nonew4q"][f] >= curly4_dev["lut6w4q"][f]).all(), f
    for name in ("lut6w4", "lut6w4q", "raw4w4", "raw4w4l"):
        assert curly4_dev[name]["mask_culls"].sum() > 0, name
    # the bit table and the codebook fetch answer every test alike: identical results per ray
    for f in ("prim", "box_tests", "tri_tests", "mask_tests", "mask_culls"):
        assert (curly4_dev["lut6w4b"][f] == curly4_dev["lut6w4"][f]).all(), f
    assert (curly4_dev["lut6w4b"]["t"].view(np.uint32) == curly4_dev["lut6w4"]["t"].view(np.uint32)).all()


# --------------------------------------------------------------------- batch64
@pytest.fixture(scope="module")
def batch64(request):
    _say(request, "batch64: generating 64 scenes")
    specs = scenes.batch_specs(64)
    return specs, [scenes.batch_scene(sp) for sp in specs]


@pytest.mark.timeout(900)
def test_batch64_graph_equals_per_scene_and_oracle(request, ctx, batch64):
    import torch
    from paper_2305_08343_amd import binding
    specs, data = batch64
    _say(request, f"batch64: build 64 scenes (raw R=6), graph launch over {sum(r.shape[0] for _, r in data)} rays")
    built = [binding.Scene(ctx, t, R=6, mode="raw") for t, _ in data]
    b = binding.Batch(ctx, [(s, r) for s, (_, r) in zip(built, data)], graph=True)
    b.launch()
    b.launch()
    torch.cuda.synchronize()
    for k, s in enumerate(built):
        single = s.trace(b.rays[k]).numpy()
        batched = b.results(k).numpy()
        for f in ("prim", "box_tests", "tri_tests", "mask_tests", "mask_culls"):
            assert (single[f] == batched[f]).all(), (k, f)
        assert (single["t"].view(np.uint32) == batched["t"].view(np.uint32)).all()
    nt = oracle.cpu_threads()
    for k in (0, 1, 2):  # one scene of each kind against the oracle
        t, r = data[k]
        _say(request, f"batch64: oracle check of scene {k} ({specs[k].kind}, {t.shape[0]} tris)")
        bvh = oracle.bvh_build(t)
        ob, delta = oracle.default_bounds(t)
        sel = slice(None, None, 8)
        ora = oracle.trace(t, bvh, r[sel], mode="raw", R=6, masks=oracle.object_masks(t, bvh, 6, delta, nthreads=nt),
                           origin_bound=ob, nthreads=nt)
        _compare(b.results(k).numpy(), ora, sel)
    b.close()
    for s in built:
        s.close()
