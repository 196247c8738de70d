"""The seeded input generators (no GPU): sizes of the benchmark workloads, determinism per seed,
float32 layouts, and the geometric facts the input recipe states (unit directions, tmin = 0,
tmax = +inf, bounce origins pushed off their triangle's plane along its normal)."""
import numpy as np
import pytest

from paper_2305_08343_amd import scenes


def _unit_dirs(rays):
    d = rays[:, 4:7].astype(np.float64)
    return np.abs(np.linalg.norm(d, axis=1) - 1.0).max()


def test_workload_sizes():
    assert scenes.scene_small(0).shape == (4096, 3, 3)
    assert scenes.rays_small().shape == (65536, 8)
    hair = scenes.scene_hair_1m(1)
    assert hair.shape == (1_000_002, 3, 3) and hair.dtype == np.float32
    # the 12M-triangle configuration: 120,000 strands x 50 segments x 2 triangles (checked on 100 strands)
    assert scenes.scene_curly_12m(2, n_strands=100).shape == (100 * 50 * 2, 3, 3)
    assert len(scenes.batch_specs()) == 64 and len(scenes.placement_specs()) == 200


@pytest.mark.parametrize("gen", [
    lambda s: scenes.strands_random_walk(s, 8, 8, 2e-3),
    lambda s: scenes.strands_helical(s, 10, 6, 1e-3, 5e-3, 0.25, (0, 0, 0), (1, 1, 1)),
    lambda s: scenes.thin_quads(s, 20),
    lambda s: scenes.isotropic_tris(s, 30),
    lambda s: scenes.micro_scene(s, 40),
    lambda s: scenes.random_rays(50, s),
])
def test_generators_are_deterministic_per_seed(gen):
    a, b, c = gen(3), gen(3), gen(4)
    assert a.dtype == np.float32
    assert np.isfinite(a[:, :7] if a.ndim == 2 else a).all()  # rays may carry tmax = +inf
    assert a.tobytes() == b.tobytes()
    assert a.tobytes() != c.tobytes()


def test_pinhole_rays():
    r = scenes.pinhole_rays(64, 32)
    assert r.shape == (64 * 32, 8) and r.dtype == np.float32
    assert (r[:, 0:3] == np.float32([0.5, 0.5, 2.2])).all()
    assert (r[:, 3] == 0).all() and np.isinf(r[:, 7]).all()
    assert _unit_dirs(r) < 1e-6
    # the centre of the image looks at (0.5, 0.5, 0.5): direction close to -z
    mid = r[16 * 64 + 32, 4:7]
    assert mid[2] < -0.99


def test_surface_bounce_rays_leave_the_surface():
    tris = scenes.strands_helical(5, 50, 10, 1e-3, 5e-3, 0.25, (0, 0, 0), (1, 1, 1))
    r = scenes.surface_bounce_rays(tris, 4000, 7)
    assert r.shape == (4000, 8) and r.dtype == np.float32
    assert (r[:, 3] == 0).all() and np.isinf(r[:, 7]).all()
    assert _unit_dirs(r) < 1e-6
    # every origin is within the offset (2^-16) of the plane of some triangle, on the side the direction
    # leaves into: check against the closest triangle plane among all triangles
    v = tris.astype(np.float64)
    n = np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0])
    ln = np.linalg.norm(n, axis=1)
    ok = ln > 0
    n, v0 = n[ok] / ln[ok, None], v[ok, 0]
    o = r[:64, 0:3].astype(np.float64)
    d = r[:64, 4:7].astype(np.float64)
    signed = np.einsum("rtk,tk->rt", o[:, None, :] - v0[None], n)
    near = np.abs(np.abs(signed) - 2.0 ** -16).min(axis=1)
    assert (near < 1e-6).all()
    k = np.abs(np.abs(signed) - 2.0 ** -16).argmin(axis=1)
    side = np.sign(signed[np.arange(64), k])
    assert (np.einsum("rk,rk->r", d, n[k]) * side >= -1e-6).all()


def test_hair_rays_are_primary_then_bounce():
    tris = scenes.scene_hair_1m(1)
    r = scenes.rays_hair_1m(tris, 1, width=32, height=16)
    assert r.shape == (2 * 32 * 16, 8)
    prim = scenes.pinhole_rays(32, 16)
    assert r[:512].tobytes() == prim.tobytes()
    assert not (r[512:, 0:3] == prim[0, 0:3]).all(axis=1).any()


def test_lattice_and_segment_scenes():
    lat = scenes.lattice_copies(3)
    assert lat.shape == (16 * 16 * 8, 3, 3) and lat.dtype == np.float32
    # copies of a shape differ by lattice steps of 1/8
    assert np.allclose(lat[3] - lat[0], lat[3, 0] - lat[0, 0])
    seg = scenes.segment_rows(0)
    e1 = seg[:, 1] - seg[:, 0]
    e2 = seg[:, 2] - seg[:, 0]
    assert (np.cross(e1, e2) == 0).all()           # zero area
    assert (e1[:, 1:] == 0).all() and (e1[:, 0] > 0).all()  # along +x
