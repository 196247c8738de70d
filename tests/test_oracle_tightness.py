"""Tightness references of the ray mask (Sect. 4.1 ideal culling, Sect. 4.2
R_ray = 2R), analysis only.

Pins:
* 2R table: every entry lies inside the R-table entry of the coarse cells
  that hold its fine cells, is symmetric in (entry, exit), and a segment that
  stays in one fine cell maps to that cell's coarse voxel;
* ideal mask: contains every voxel holding a densely sampled point of the
  segment, and only voxels at float64 distance ~0 from the segment (closest
  point of the segment to each voxel box, a different computation);
* culling with either reference never changes the hit, and the aggregate
  test count orders ideal <= 2R table <= R table <= no culling.
The Table 1 analog on a sample of the 1M-triangle hair workload is printed
(-s) for the design notes.
"""
import numpy as np
import pytest

import oracle
from paper_2305_08343_amd import scenes


def _bits(m, R):
    return oracle.mask_bits(np.asarray(m, np.uint64)[None], R)[0].astype(bool)


def test_lut2_inside_coarse_table_r4():
    R, F = 4, 8
    l2 = oracle.raymask_lut2(R)
    l1 = oracle.raymask_lut(R)
    keys = np.arange(F ** 6)
    e = np.stack([(keys // F ** 2) % F, (keys // F) % F, keys % F], 1)
    b = np.stack([(keys // F ** 5) % F, (keys // F ** 4) % F, (keys // F ** 3) % F], 1)
    cb, ce = b // 2, e // 2
    ck = ((((cb[:, 0] * R + cb[:, 1]) * R + cb[:, 2]) * R + ce[:, 0]) * R + ce[:, 1]) * R + ce[:, 2]
    assert ((l2 & ~l1[ck]) == 0).all()
    swap = ((((e[:, 0] * F + e[:, 1]) * F + e[:, 2]) * F + b[:, 0]) * F + b[:, 1]) * F + b[:, 2]
    assert (l2 == l2[swap]).all()
    same = (b == e).all(1)
    for k in np.flatnonzero(same)[::37]:
        x, y, z = cb[k]
        want = np.uint64(1) << np.uint64(x + R * y + R * R * z)
        assert l2[k, 0] == want
    # strictly tighter somewhere
    assert (l2 != l1[ck]).any()


def _segment_box_distance(o, d, t0, t1, lo, hi, n=2001):
    """Closest distance from the segment to the box, by minimizing over a fine
    parameter grid refined around the best sample (float64)."""
    ts = np.linspace(t0, t1, n)
    p = o[None] + ts[:, None] * d[None]
    q = np.clip(p, lo, hi)
    dist = np.linalg.norm(p - q, axis=1)
    k = int(np.argmin(dist))
    a, b = ts[max(k - 1, 0)], ts[min(k + 1, n - 1)]
    ts = np.linspace(a, b, n)
    p = o[None] + ts[:, None] * d[None]
    return np.linalg.norm(p - np.clip(p, lo, hi), axis=1).min()


@pytest.mark.parametrize("R", [4, 6])
def test_ideal_mask_sampled_and_distance_bounds(R):
    rng = np.random.default_rng(R)
    for _ in range(60):
        lo = rng.uniform(-1, 0, 3).astype(np.float32)
        hi = (lo + rng.uniform(0.2, 2.0, 3)).astype(np.float32)
        o = rng.uniform(-2, 2, 3).astype(np.float32)
        d = rng.normal(size=3).astype(np.float32)
        d[rng.random(3) < 0.15] = 0.0
        if not d.any():
            d[0] = 1.0
        t0, t1 = np.float32(rng.uniform(-1, 1)), np.float32(rng.uniform(1, 3))
        m = _bits(oracle.ideal_mask(np.concatenate([lo, hi]), o, d, t0, t1, R), R)
        o64, d64 = o.astype(np.float64), d.astype(np.float64)
        ext = hi.astype(np.float64) - lo.astype(np.float64)
        edges = [lo[j] + (np.arange(R + 1) * ext[j]) / R for j in range(3)]
        # lower bound: voxels holding sampled points strictly inside a voxel
        ts = np.linspace(t0, t1, 4001)
        pts = o64[None] + ts[:, None] * d64[None]
        idx = [np.searchsorted(edges[j], pts[:, j], side="right") - 1 for j in range(3)]
        inside = np.all([(idx[j] >= 0) & (idx[j] < R) for j in range(3)], axis=0)
        for x, y, z in zip(idx[0][inside], idx[1][inside], idx[2][inside]):
            assert m[x + R * y + R * R * z]
        # upper bound: every voxel in the mask is (numerically) touched by the segment
        for bit in np.flatnonzero(m):
            x, y, z = bit % R, (bit // R) % R, bit // (R * R)
            vlo = np.array([edges[0][x], edges[1][y], edges[2][z]])
            vhi = np.array([edges[0][x + 1], edges[1][y + 1], edges[2][z + 1]])
            assert _segment_box_distance(o64, d64, float(t0), float(t1), vlo, vhi) < 1e-6 * (1 + np.abs(ext).max())


def _tightness(tris, rays, R, kinds, nt=0):
    bvh = oracle.bvh_build(tris)
    ob, delta = oracle.default_bounds(tris)
    masks = oracle.object_masks(tris, bvh, R, delta, nthreads=nt)
    none = oracle.trace(tris, bvh, rays, origin_bound=ob, nthreads=nt)
    out = {"none": none}
    for k in kinds:
        out[k] = oracle.trace(tris, bvh, rays, mode="raw", R=R, masks=masks, origin_bound=ob, ray_masks=k,
                              nthreads=nt)
        assert (out[k].prim == none.prim).all() and (out[k].t.view(np.uint32) == none.t.view(np.uint32)).all()
    return {k: float((h.box_tests.astype(np.float64) + h.tri_tests).sum()) for k, h in out.items()}


@pytest.mark.parametrize("R", [4, 6])
def test_tightness_order_small_scene(small_scene, R):
    tris, rays = small_scene
    kinds = ("lut", "ideal", "lut2r") if R == 4 else ("lut", "ideal")
    t = _tightness(tris, rays, R, kinds)
    assert t["ideal"] <= t["lut"] <= t["none"]
    if "lut2r" in t:
        assert t["ideal"] <= t["lut2r"] <= t["lut"]


@pytest.mark.slow
def test_table1_analog_hair_sample(capsys):
    tris = scenes.scene_hair_1m(1)
    rays = scenes.rays_hair_1m(tris, 1)[::64]
    rows = []
    for R, kinds in ((4, ("lut", "lut2r", "ideal")), (6, ("lut", "ideal"))):
        t = _tightness(tris, rays, R, kinds, nt=oracle.cpu_threads())
        assert t["ideal"] <= t["lut"] <= t["none"]
        rows.append((R, {k: t[k] / t["none"] for k in kinds}))
    with capsys.disabled():
        print(f"\n[tightness] hair_1m, every 64th ray ({rays.shape[0]}): tests ratio vs unculled")
        for R, r in rows:
            print(f"[tightness] R={R}: " + ", ".join(f"{k} {v:.4f}" for k, v in r.items()))
