"""The library's host BVH builder (sequential and multi-threaded paths) equals
the oracle's build bit for bit (CPU only; no device)."""
import time

import numpy as np
import pytest

import oracle
from paper_2305_08343_amd import binding, scenes


def _same(lib, ob):
    assert lib["n_inner"] == ob.n_inner and lib["depth"] == ob.depth and lib["root"] == ob.root
    assert (lib["cbox"].view(np.uint32) == ob.cbox.view(np.uint32)).all()
    assert (lib["cref"] == ob.cref).all() and (lib["range"] == ob.range).all()
    assert (lib["perm"] == ob.perm).all()


@pytest.mark.parametrize("seed", range(20))
def test_micro_scenes(seed):
    t = scenes.micro_scene(seed, 1 + (seed * 7) % 64)
    _same(binding.bvh_build_host(t), oracle.bvh_build(t))


def test_small_scene_and_options(small_scene):
    t, _ = small_scene
    _same(binding.bvh_build_host(t), oracle.bvh_build(t))
    for leaf, bins in ((1, 8), (2, 2), (3, 256)):
        _same(binding.bvh_build_host(t, leaf_max=leaf, bins=bins), oracle.bvh_build(t, leaf_max=leaf, bins=bins))


def test_million_triangles_parallel_path():
    """1M triangles: large subtrees are built on worker threads and spliced."""
    t = scenes.scene_hair_1m(1)
    t0 = time.time()
    lib = binding.bvh_build_host(t)
    dt = time.time() - t0
    _same(lib, oracle.bvh_build(t))
    print(f"host BVH build of {t.shape[0]} tris: {dt:.2f} s")


def test_errors_and_empty():
    e = binding.bvh_build_host(np.zeros((0, 3, 3), np.float32))
    assert e["n_inner"] == 0 and e["root"] == 0xFFFFFFFF
    with pytest.raises(binding.SubcullError) as ex:
        binding.bvh_build_host(scenes.scene_small(0), depth_cap=3)
    assert ex.value.status == 4
    bad = scenes.scene_small(0)
    bad[3, 2, 1] = np.inf
    with pytest.raises(binding.SubcullError) as ex:
        binding.bvh_build_host(bad)
    assert ex.value.status == 1
