"""GPU parity of the approximate object masks (Sect. 3.2.1, Alg. 2) against the
oracle: every child-slot mask bit for bit at L = 1, 2, 3, 5 and R = 4, 6
(small strand scene, micro scenes, the 1M-triangle hair scene at L = 3), and
per-ray traversal results with those masks on both BVH widths."""
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


def _compare(dev, ora):
    for k, o in (("prim", ora.prim), ("box_tests", ora.box_tests), ("tri_tests", ora.tri_tests),
                 ("mask_tests", ora.mask_tests), ("mask_culls", ora.mask_culls)):
        bad = np.flatnonzero(dev[k] != o)
        assert bad.size == 0, f"{k}: {bad.size} rays differ, first {bad[:5]}"
    assert (dev["t"].view(np.uint32) == ora.t.view(np.uint32)).all()


@pytest.mark.parametrize("R", [4, 6])
@pytest.mark.parametrize("L", [1, 2, 3, 5])
def test_masks_and_trace_small_scene(ctx, small_scene, small_oracle, R, L):
    from paper_2305_08343_amd import binding
    tris, rays = small_scene
    bvh = small_oracle["bvh"]
    print(f"[gpu-approx] small scene R={R} L={L}", flush=True)
    ref = oracle.approx_masks(tris, bvh, R, small_oracle["delta"], L)
    s = binding.Scene(ctx, tris, R=R, mode="raw", approx_levels=L)
    assert (s.export()["masks"] == ref).all()
    dev = s.trace(rays).numpy()
    s.close()
    _compare(dev, oracle.trace(tris, bvh, rays, mode="raw", R=R, masks=ref,
                               origin_bound=small_oracle["origin_bound"]))
    s4 = binding.Scene(ctx, tris, R=R, mode="raw", approx_levels=L, width=4)
    dev4 = s4.trace(rays).numpy()
    s4.close()
    _compare(dev4, oracle.trace4(tris, bvh, oracle.bvh4_collapse(bvh), rays, mode="raw", R=R, masks=ref,
                                 origin_bound=small_oracle["origin_bound"]))


@pytest.mark.parametrize("seed", range(12))
def test_micro_scenes(ctx, seed):
    from paper_2305_08343_amd import binding
    tris = scenes.micro_scene(seed, 1 + (seed * 11) % 64)
    bvh = oracle.bvh_build(tris)
    _, delta = oracle.default_bounds(tris)
    R, L = (6, 1 + seed % 3) if seed % 2 else (4, 1 + seed % 3)
    print(f"[gpu-approx] micro scene {seed} R={R} L={L}", flush=True)
    s = binding.Scene(ctx, tris, R=R, mode="raw", approx_levels=L)
    got = s.export()["masks"]
    s.close()
    assert (got == oracle.approx_masks(tris, bvh, R, delta, L)).all()


@pytest.mark.timeout(600)
def test_hair_1m_level_3(ctx):
    from paper_2305_08343_amd import binding
    print("[gpu-approx] hair_1m R=6 L=3: generate, oracle masks", flush=True)
    tris = scenes.scene_hair_1m(1)
    bvh = oracle.bvh_build(tris)
    _, delta = oracle.default_bounds(tris)
    ref = oracle.approx_masks(tris, bvh, 6, delta, 3)
    print("[gpu-approx] hair_1m R=6 L=3: device build", flush=True)
    s = binding.Scene(ctx, tris, R=6, mode="raw", approx_levels=3)
    got = s.export()["masks"]
    s.close()
    assert (got == ref).all()
