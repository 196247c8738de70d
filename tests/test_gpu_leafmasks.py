"""Masks on leaf slots only (build option mask_slots = leaves) on the GPU: the
device masks equal the oracle's leaf_slot_masks of its exact masks, and every
per-ray result -- hit, t bits, box / triangle / mask counts, culled and
unculled -- equals the oracle's trace with those masks, on the binary and the
4-wide BVH, raw and LUT-compressed."""
import numpy as np
import pytest

import oracle
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


@pytest.mark.parametrize("mode,R,K,width", [("raw", 6, 0, 2), ("raw", 4, 0, 2), ("raw", 6, 0, 4), ("raw", 4, 0, 4),
                                            ("lut", 6, 4096, 4), ("lut", 4, 256, 2)])
def test_leaf_slot_masks_bit_exact(ctx, small_scene, small_oracle, mode, R, K, width):
    from paper_2305_08343_amd import binding
    tris, rays = small_scene
    rays = np.concatenate([rays, _aimed(tris, 20011, 53)])
    bvh = small_oracle["bvh"]
    lm = oracle.leaf_slot_masks(small_oracle[f"masks{R}"], bvh, R)
    print(f"[gpu-leaf] {mode} R={R} K={K} width={width}", flush=True)
    s = binding.Scene(ctx, tris, R=R, mode=mode, K=K or 4096, width=width, mask_slots="leaves")
    exp = s.export()
    assert (exp["masks"] == lm).all()
    kw = dict(origin_bound=small_oracle["origin_bound"])
    if mode == "raw":
        kw.update(mode="raw", R=R, masks=lm)
    else:
        cb, idx = oracle.compress(lm, bvh.slot_boxes(), R, K)
        assert (exp["codebook"] == cb).all() and (exp["cidx"] == idx).all()
        kw.update(mode="lut", R=R, codebook=cb, cidx=idx)
    b4 = oracle.bvh4_collapse(bvh) if width == 4 else None
    for cull in (True, False):
        ora = (oracle.trace(tris, bvh, rays, cull=cull, **kw) if width == 2
               else oracle.trace4(tris, bvh, b4, rays, cull=cull, **kw))
        _compare(s.trace(rays, cull=cull).numpy(), ora)
    s.close()


def test_bad_mask_slots_rejected(ctx, small_scene):
    from paper_2305_08343_amd import binding
    with pytest.raises(ValueError):
        binding.Scene(ctx, small_scene[0], mask_slots="inner")


@pytest.mark.parametrize("seed", range(16))
def test_leaf_slot_masks_micro_scenes(ctx, seed):
    from paper_2305_08343_amd import binding, scenes
    n = 1 + (seed * 13) % 64
    tris = scenes.micro_scene(seed, n)
    rays = np.concatenate([_aimed(tris, 300, seed), scenes.random_rays(100, seed)])
    bvh = oracle.bvh_build(tris)
    b4 = oracle.bvh4_collapse(bvh)
    ob, delta = oracle.default_bounds(tris)
    print(f"[gpu-leaf] micro scene {seed} ({n} tris)", flush=True)
    for R in (4, 6):
        lm = oracle.leaf_slot_masks(oracle.object_masks(tris, bvh, R, delta), bvh, R)
        for width in (2, 4):
            s = binding.Scene(ctx, tris, R=R, mode="raw", width=width, mask_slots="leaves")
            ora = (oracle.trace(tris, bvh, rays, mode="raw", R=R, masks=lm, origin_bound=ob) if width == 2 else
                   oracle.trace4(tris, bvh, b4, rays, mode="raw", R=R, masks=lm, origin_bound=ob))
            _compare(s.trace(rays).numpy(), ora)
            s.close()
