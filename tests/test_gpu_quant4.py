"""GPU parity of 4-wide scenes with quantised child boxes (8-bit steps from
the node's corner, rounded outward; a node layout of this library, not of the
paper) against the oracle's decoded BVH4: the decoded boxes and the binary
slot boxes, masks built on them, and per ray hit id, t, box / triangle / mask
counts in modes NONE, RAW (every slot and leaf slots only) and LUT (codebook
in LDS and through the caches, and the 2-D bit table), culled and in
shadow mode, in every launch shape, plus micro scenes, degenerate inputs and
extreme scales (a flat scene, scenes scaled by 1e15 and 1e-8). Hits also equal
those of the exact-box scene."""
import numpy as np
import pytest

import oracle
from paper_2305_08343_amd import scenes
from tests.test_gpu_bvh4 import _aimed, _compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_2305_08343_amd import binding
    c = binding.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def quant_oracle(small_scene, small_oracle):
    """Decoded 4-wide BVH, binary BVH with the decoded slot boxes, masks on them."""
    tris, _ = small_scene
    bvh = small_oracle["bvh"]
    b4 = oracle.bvh4_collapse(bvh)
    d4 = oracle.decoded_bvh4(b4, oracle.quantise4(b4))
    bq = oracle.with_slot_boxes(bvh, d4)
    delta = small_oracle["delta"]
    return {"b4": b4, "d4": d4, "bq": bq,
            "masks4": oracle.object_masks(tris, bq, 4, delta), "masks6": oracle.object_masks(tris, bq, 6, delta)}


def test_decoded_boxes_and_slot_boxes_match_oracle(ctx, small_scene, small_oracle, quant_oracle):
    from paper_2305_08343_amd import binding
    tris, _ = small_scene
    d4, bq = quant_oracle["d4"], quant_oracle["bq"]
    for mode in ("none", "raw"):
        print(f"[gpu-quant4] export, mode {mode}", flush=True)
        s = binding.Scene(ctx, tris, R=6, mode=mode, width=4, quantise=True)
        assert s.info["width"] == 4 and s.info["n_nodes"] == d4.n4 and s.info["node_bytes"] == 64
        e4, e = s.export4(), s.export()
        s.close()
        assert (e4["box4"].view(np.uint32) == d4.box4.view(np.uint32)).all()
        assert (e4["ref4"] == d4.ref4).all() and (e4["src4"] == d4.src4).all()
        assert (e["cbox"].view(np.uint32) == bq.cbox.view(np.uint32)).all()
        if mode == "raw":
            assert (e["masks"] == quant_oracle["masks6"]).all()
    # the decoded boxes really differ from the exact ones
    used = d4.ref4 != oracle.EMPTY_REF
    assert (d4.box4[used] != quant_oracle["b4"].box4[used]).any()


@pytest.mark.parametrize("mode,R,slots", [("none", 6, "all"), ("raw", 6, "all"), ("raw", 4, "all"),
                                          ("raw", 6, "leaves"), ("raw", 4, "leaves")])
def test_trace_bit_exact(ctx, small_scene, small_oracle, quant_oracle, mode, R, slots):
    import torch
    from paper_2305_08343_amd import binding
    tris, rays = small_scene
    rays = np.concatenate([rays, _aimed(tris, 30011, 51)])
    bq, d4 = quant_oracle["bq"], quant_oracle["d4"]
    kw = dict(origin_bound=small_oracle["origin_bound"])
    if mode == "raw":
        m = quant_oracle[f"masks{R}"]
        if slots == "leaves":
            m = oracle.leaf_slot_masks(m, bq, R)
        kw.update(mode="raw", R=R, masks=m)
    print(f"[gpu-quant4] trace {mode} R={R} slots={slots}", flush=True)
    s = binding.Scene(ctx, tris, R=R, mode=mode, width=4, quantise=True, mask_slots=slots)
    for cull in (True, False):
        _compare(s.trace(rays, cull=cull).numpy(), oracle.trace4(tris, bq, d4, rays, cull=cull, **kw))
    if mode != "none":
        fp = torch.zeros(2 * bq.n_inner, dtype=torch.int32, device="cuda:0")
        dev = s.trace(rays, cull=False, shadow=True, slot_fp=fp).numpy()
        ora = oracle.trace4(tris, bq, d4, rays, cull=False, shadow=True, **kw)
        _compare(dev, ora)
        assert (fp.cpu().numpy().view(np.uint32) == ora.slot_fp).all() and ora.slot_fp.sum() > 0
    s.close()


def test_hits_equal_exact_box_scene(ctx, small_scene):
    from paper_2305_08343_amd import binding
    tris, rays = small_scene
    rays = np.concatenate([rays, _aimed(tris, 20000, 52)])
    print("[gpu-quant4] hits of quantised and exact boxes", flush=True)
    for mode in ("none", "raw"):
        a = binding.Scene(ctx, tris, R=6, mode=mode, width=4)
        b = binding.Scene(ctx, tris, R=6, mode=mode, width=4, quantise=True)
        ha, hb = a.trace(rays).numpy(), b.trace(rays).numpy()
        a.close()
        b.close()
        assert (ha["prim"] == hb["prim"]).all() and (ha["t"].view(np.uint32) == hb["t"].view(np.uint32)).all()
        assert (ha["prim"] != oracle.NO_HIT).mean() > 0.2


@pytest.mark.parametrize("seed", range(12))
def test_micro_scenes(ctx, seed):
    from paper_2305_08343_amd import binding
    n = 1 + (seed * 17) % 64
    tris = scenes.micro_scene(seed, n)
    rays = np.concatenate([_aimed(tris, 300, seed), scenes.random_rays(100, seed)])
    bvh = oracle.bvh_build(tris)
    b4 = oracle.bvh4_collapse(bvh)
    d4 = oracle.decoded_bvh4(b4, oracle.quantise4(b4))
    bq = oracle.with_slot_boxes(bvh, d4)
    ob, delta = oracle.default_bounds(tris)
    bp, bt = oracle.brute_closest(tris, rays)
    print(f"[gpu-quant4] micro scene {seed} ({n} tris)", flush=True)
    for R in (4, 6):
        s = binding.Scene(ctx, tris, R=R, mode="raw", width=4, quantise=True)
        masks = oracle.object_masks(tris, bq, R, delta)
        dev = s.trace(rays).numpy()
        s.close()
        _compare(dev, oracle.trace4(tris, bq, d4, rays, mode="raw", R=R, masks=masks, origin_bound=ob))
        assert (dev["prim"] == bp).all() and (dev["t"].view(np.uint32) == bt.view(np.uint32)).all()


def test_every_launch_shape(ctx, small_scene, small_oracle, quant_oracle):
    from paper_2305_08343_amd import binding
    tris, rays = small_scene
    rays = np.concatenate([rays, _aimed(tris, 20000, 53)])
    bq, d4 = quant_oracle["bq"], quant_oracle["d4"]
    ora = oracle.trace4(tris, bq, d4, rays, mode="raw", R=6, masks=quant_oracle["masks6"],
                        origin_bound=small_oracle["origin_bound"])
    s = binding.Scene(ctx, tris, R=6, mode="raw", width=4, quantise=True)
    try:
        for block, stack in ((256, 8), (128, 8), (256, 12), (256, 4), (128, 16)):
            for chunk, parts, waves, sort, gather, refill in ((1, 8, 0, 0, 0, 1), (2, 1, 6, 1, 12, 12)):
                print(f"[gpu-quant4] tune {block} {stack} {chunk} {parts} {waves} {sort} {gather} {refill}",
                      flush=True)
                ctx.set_tune(block, stack, chunk, parts, waves, sort, 0, gather, refill)
                _compare(s.trace(rays).numpy(), ora)
    finally:
        ctx.set_tune()
        s.close()


def test_degenerate_inputs_and_rejections(ctx, small_scene):
    from paper_2305_08343_amd import binding
    print("[gpu-quant4] empty scene, single leaf, rejected combinations", flush=True)
    rays = scenes.random_rays(1000, 3)
    s = binding.Scene(ctx, np.zeros((0, 3, 3), np.float32), mode="raw", width=4, quantise=True)
    d = s.trace(rays).numpy()
    s.close()
    assert (d["prim"] == oracle.NO_HIT).all() and (d["box_tests"] == 0).all()
    t = scenes.micro_scene(2, 3)
    bvh = oracle.bvh_build(t)
    s = binding.Scene(ctx, t, mode="raw", width=4, quantise=True)
    assert s.info["n_nodes"] == 0
    _compare(s.trace(rays).numpy(), oracle.trace4(t, bvh, oracle.bvh4_collapse(bvh), rays), masks=False)
    s.close()
    tris, _ = small_scene
    for kw in (dict(mode="raw", width=2), dict(mode="sparse", placement=np.ones(2, np.uint8), width=4)):
        with pytest.raises(binding.SubcullError):
            binding.Scene(ctx, tris, quantise=True, **kw)


@pytest.mark.parametrize("name", ["flat", "huge", "tiny"])
def test_extreme_scales_bit_exact(ctx, name):
    """A flat scene (zero extent in z: the smallest step exponent) and scenes scaled by 1e15 and
    1e-8, plain and with 216-bit masks on the decoded boxes."""
    from paper_2305_08343_amd import binding
    from tests.test_oracle_quant4 import extreme_case
    tris, rays = extreme_case(name)
    bvh = oracle.bvh_build(tris)
    b4 = oracle.bvh4_collapse(bvh)
    d4 = oracle.decoded_bvh4(b4, oracle.quantise4(b4))
    bq = oracle.with_slot_boxes(bvh, d4)
    ob, delta = oracle.default_bounds(tris)
    print(f"[gpu-quant4] extreme scale {name}", flush=True)
    for mode in ("none", "raw"):
        s = binding.Scene(ctx, tris, R=6, mode=mode, width=4, quantise=True)
        e4 = s.export4()
        dev = s.trace(rays).numpy()
        s.close()
        assert (e4["box4"].view(np.uint32) == d4.box4.view(np.uint32)).all()
        kw = dict(origin_bound=ob)
        if mode == "raw":
            kw.update(mode="raw", R=6, masks=oracle.object_masks(tris, bq, 6, delta))
        _compare(dev, oracle.trace4(tris, bq, d4, rays, **kw), masks=(mode == "raw"))


@pytest.mark.parametrize("L", [1, 3])
def test_approximate_masks_on_decoded_boxes(ctx, small_scene, small_oracle, quant_oracle, L):
    """Alg. 2 masks of a quantised scene are built on the decoded slot boxes, like exact ones."""
    from paper_2305_08343_amd import binding
    tris, rays = small_scene
    bq, d4 = quant_oracle["bq"], quant_oracle["d4"]
    print(f"[gpu-quant4] approximate masks L={L}", flush=True)
    ref = oracle.approx_masks(tris, bq, 6, small_oracle["delta"], L)
    s = binding.Scene(ctx, tris, R=6, mode="raw", approx_levels=L, width=4, quantise=True)
    assert (s.export()["masks"] == ref).all()
    dev = s.trace(rays).numpy()
    s.close()
    _compare(dev, oracle.trace4(tris, bq, d4, rays, mode="raw", R=6, masks=ref,
                                origin_bound=small_oracle["origin_bound"]))


@pytest.mark.parametrize("R,K,bits", [(6, 4096, False), (6, 256, False), (4, 256, False), (6, 256, True)])
def test_lut_modes_bit_exact(ctx, small_scene, small_oracle, quant_oracle, R, K, bits):
    """Compressed masks of a quantised scene: codebook and indices from the masks on the decoded
    slot boxes (importance weighted by their areas), indices read from the node's last piece."""
    import torch
    from paper_2305_08343_amd import binding
    tris, rays = small_scene
    rays = np.concatenate([rays, _aimed(tris, 20011, 54)])
    bq, d4 = quant_oracle["bq"], quant_oracle["d4"]
    cb, idx = oracle.compress(quant_oracle[f"masks{R}"], bq.slot_boxes(), R, K)
    kw = dict(origin_bound=small_oracle["origin_bound"], mode="lut", R=R, codebook=cb, cidx=idx)
    print(f"[gpu-quant4] LUT R={R} K={K} bit_table={bits}", flush=True)
    s = binding.Scene(ctx, tris, R=R, mode="lut", K=K, width=4, quantise=True, bit_table=bits)
    e = s.export()
    assert (e["codebook"] == cb).all() and (e["cidx"] == idx).all()
    try:
        for cbg in (0, 1):
            ctx.set_tune(codebook=cbg)
            for cull in (True, False):
                _compare(s.trace(rays, cull=cull).numpy(), oracle.trace4(tris, bq, d4, rays, cull=cull, **kw))
    finally:
        ctx.set_tune()
    fp = torch.zeros(2 * bq.n_inner, dtype=torch.int32, device="cuda:0")
    dev = s.trace(rays, cull=False, shadow=True, slot_fp=fp).numpy()
    ora = oracle.trace4(tris, bq, d4, rays, cull=False, shadow=True, **kw)
    s.close()
    _compare(dev, ora)
    assert (fp.cpu().numpy().view(np.uint32) == ora.slot_fp).all() and ora.slot_fp.sum() > 0


@pytest.mark.parametrize("seed", range(6))
def test_lut_micro_scenes(ctx, seed):
    """Compressed masks (K = 64) on quantised micro scenes, every ray bit for bit."""
    from paper_2305_08343_amd import binding
    n = 2 + (seed * 19) % 63
    tris = scenes.micro_scene(seed + 40, n)
    rays = np.concatenate([_aimed(tris, 300, seed), scenes.random_rays(100, seed)])
    bvh = oracle.bvh_build(tris)
    b4 = oracle.bvh4_collapse(bvh)
    d4 = oracle.decoded_bvh4(b4, oracle.quantise4(b4))
    bq = oracle.with_slot_boxes(bvh, d4)
    ob, delta = oracle.default_bounds(tris)
    print(f"[gpu-quant4] LUT micro scene {seed} ({n} tris)", flush=True)
    for R in (4, 6):
        cb, idx = oracle.compress(oracle.object_masks(tris, bq, R, delta), bq.slot_boxes(), R, 64)
        s = binding.Scene(ctx, tris, R=R, mode="lut", K=64, width=4, quantise=True)
        dev = s.trace(rays).numpy()
        s.close()
        _compare(dev, oracle.trace4(tris, bq, d4, rays, mode="lut", R=R, codebook=cb, cidx=idx, origin_bound=ob))


@pytest.mark.parametrize("kind", ["low", "high"])
def test_mixed_magnitude_nodes_bit_exact(ctx, kind):
    """Child planes far smaller than the node's corner (and a greatest maximum the covering step
    cannot reach): the library's counts, decoded boxes and traces equal the oracle's, whose decoded
    boxes contain every child box."""
    from paper_2305_08343_amd import binding
    from tests.test_oracle_quant4 import mixed_magnitude_case
    tris, rays = mixed_magnitude_case(kind)
    bvh = oracle.bvh_build(tris)
    b4 = oracle.bvh4_collapse(bvh)
    d4 = oracle.decoded_bvh4(b4, oracle.quantise4(b4))
    bq = oracle.with_slot_boxes(bvh, d4)
    ob, delta = oracle.default_bounds(tris)
    print(f"[gpu-quant4] mixed magnitudes {kind}", flush=True)
    for mode in ("none", "raw"):
        s = binding.Scene(ctx, tris, R=6, mode=mode, width=4, quantise=True)
        e4 = s.export4()
        dev = s.trace(rays).numpy()
        s.close()
        assert (e4["box4"].view(np.uint32) == d4.box4.view(np.uint32)).all()
        kw = dict(origin_bound=ob)
        if mode == "raw":
            kw.update(mode="raw", R=6, masks=oracle.object_masks(tris, bq, 6, delta))
        _compare(dev, oracle.trace4(tris, bq, d4, rays, **kw), masks=(mode == "raw"))
