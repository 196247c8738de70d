"""Seeded synthetic scenes and rays (inputs only).

This module produces the triangle soups and ray batches that both the HIP
path and the CPU oracle consume. It holds none of the culling method's
arithmetic: no BVH, no voxel masks, no intersection tests. Everything is
drawn from ``numpy.random.default_rng(seed)`` in float64 and rounded to
float32 once at the end, so the same seed gives the same arrays on any
machine.

The paper evaluates on hair and architectural scenes (Sect. 4, scene figure)
that are not available here; thin, tilted, curly strands stand in for the
hair scenes (where the paper reports its largest reductions, Table 1) and
well-shaped isotropic triangles stand in for the architectural ones.

Layouts
-------
triangles : float32 [n, 3, 3]  (triangle, vertex, xyz)
rays      : float32 [m, 8]     (ox, oy, oz, tmin, dx, dy, dz, tmax)
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "strands_random_walk", "strands_helical", "ground_plane", "thin_quads",
    "isotropic_tris", "pinhole_rays", "surface_bounce_rays", "random_rays",
    "scene_small", "scene_hair_1m", "scene_curly_12m", "rays_small",
    "rays_hair_1m", "rays_curly_12m", "micro_scene", "batch_specs",
    "batch_scene", "BatchSpec",
]


# ----------------------------------------------------------------------------
# small vector helpers (float64)
# ----------------------------------------------------------------------------
def _unit(v: np.ndarray) -> np.ndarray:
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _perp_basis(t: np.ndarray):
    """Two unit vectors orthogonal to the unit vectors ``t`` [..., 3]."""
    pick = np.where(np.abs(t[..., :1]) < 0.9, np.array([1.0, 0.0, 0.0]),
                    np.array([0.0, 1.0, 0.0]))
    e1 = _unit(np.cross(t, pick))
    e2 = np.cross(t, e1)
    return e1, e2


def _rotate(v, axis, ang):
    """Rodrigues rotation of ``v`` about unit ``axis`` by ``ang`` radians."""
    c = np.cos(ang)[..., None]
    s = np.sin(ang)[..., None]
    return v * c + np.cross(axis, v) * s + axis * np.sum(axis * v, -1, keepdims=True) * (1 - c)


def _uniform_sphere(rng, n):
    z = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2 * math.pi, n)
    r = np.sqrt(np.maximum(0.0, 1 - z * z))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], -1)


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------
def strands_random_walk(seed: int, n_strands: int = 128, n_seg: int = 32,
                        width: float = 2e-3, length: float = 0.3,
                        bend_sigma: float = 0.15, twist: float = 0.1) -> np.ndarray:
    """Curved ribbon strands, one triangle per segment, inside [0,1]^3.

    Each strand starts uniformly in [0.1, 0.9]^3 with a direction uniform on
    the sphere; every step bends the direction by N(0, bend_sigma) radians
    about a random perpendicular axis, and points leaving the unit cube are
    reflected back. Segment k gives the triangle (c_k + w/2 b_k,
    c_k - w/2 b_k, c_{k+1}) where b_k is a slowly twisting binormal.
    """
    rng = np.random.default_rng(seed)
    seg = length / n_seg
    p = rng.uniform(0.1, 0.9, (n_strands, 3))
    d = _uniform_sphere(rng, n_strands)
    b = _unit(np.cross(d, _uniform_sphere(rng, n_strands)))
    cs, bs = [p.copy()], [b.copy()]
    for _ in range(n_seg):
        ax = _unit(np.cross(d, rng.normal(size=(n_strands, 3))))
        d = _unit(_rotate(d, ax, rng.normal(0.0, bend_sigma, n_strands)))
        p = p + seg * d
        lo, hi = p < 0.0, p > 1.0
        p = np.where(lo, -p, np.where(hi, 2.0 - p, p))
        d = np.where(lo | hi, -d, d)
        b = _rotate(b, d, np.full(n_strands, twist))
        b = _unit(b - d * np.sum(b * d, -1, keepdims=True))
        cs.append(p.copy())
        bs.append(b.copy())
    c = np.stack(cs, 1)  # [S, K+1, 3]
    bb = np.stack(bs, 1)
    half = 0.5 * width
    tri = np.stack([c[:, :-1] + half * bb[:, :-1], c[:, :-1] - half * bb[:, :-1], c[:, 1:]], 2)
    return tri.reshape(-1, 3, 3).astype(np.float32)


def strands_helical(seed: int, n_strands: int, n_seg: int, width: float, curl: float,
                    length: float, root_lo, root_hi, axis=(0.0, 1.0, 0.0),
                    max_tilt_deg: float = 60.0, seg_per_turn: float = 8.0) -> np.ndarray:
    """Curly ribbon strands, two triangles (one quad) per segment.

    The centre line of strand i is root + s * L * base + curl * (cos(phi) e1 +
    sin(phi) e2) with phi advancing 2*pi per ``seg_per_turn`` segments; the
    base direction is tilted up to ``max_tilt_deg`` from ``axis`` (uniform in
    angle, uniform azimuth). The ribbon binormal is tangent x radial, so the
    ribbon plane twists with the helix and is diagonal to all three axes.
    """
    rng = np.random.default_rng(seed)
    axis = _unit(np.asarray(axis, np.float64))
    root = rng.uniform(np.asarray(root_lo, np.float64), np.asarray(root_hi, np.float64),
                       (n_strands, 3))
    theta = np.deg2rad(rng.uniform(0.0, max_tilt_deg, n_strands))
    az = rng.uniform(0.0, 2 * math.pi, n_strands)
    a1, a2 = _perp_basis(np.broadcast_to(axis, (n_strands, 3)))
    base = (np.cos(theta)[:, None] * axis + np.sin(theta)[:, None] *
            (np.cos(az)[:, None] * a1 + np.sin(az)[:, None] * a2))
    e1, e2 = _perp_basis(base)
    phase = rng.uniform(0.0, 2 * math.pi, n_strands)
    k = np.arange(n_seg + 1, dtype=np.float64)
    phi = phase[:, None] + 2 * math.pi * k[None, :] / seg_per_turn
    radial = np.cos(phi)[..., None] * e1[:, None] + np.sin(phi)[..., None] * e2[:, None]
    s = (k / n_seg)[None, :, None]
    c = root[:, None] + s * length * base[:, None] + curl * radial  # [S, K+1, 3]
    tan = np.empty_like(c)
    tan[:, :-1] = c[:, 1:] - c[:, :-1]
    tan[:, -1] = tan[:, -2]
    bn = _unit(np.cross(_unit(tan), radial))
    half = 0.5 * width
    pa, pb = c + half * bn, c - half * bn
    tri = np.empty((n_strands, n_seg, 2, 3, 3), np.float32)  # rounded once on assignment
    tri[:, :, 0, 0], tri[:, :, 0, 1], tri[:, :, 0, 2] = pa[:, :-1], pb[:, :-1], pa[:, 1:]
    tri[:, :, 1, 0], tri[:, :, 1, 1], tri[:, :, 1, 2] = pb[:, :-1], pb[:, 1:], pa[:, 1:]
    return tri.reshape(-1, 3, 3)


def ground_plane(y: float = 0.0, lo: float = -1.0, hi: float = 2.0) -> np.ndarray:
    """Two triangles covering the square [lo, hi]^2 of the plane y = const."""
    a, b, c, d = (lo, y, lo), (hi, y, lo), (hi, y, hi), (lo, y, hi)
    return np.array([[a, b, c], [a, c, d]], np.float32)


def thin_quads(seed: int, n_quads: int, length: float = 0.02, width: float = 5e-4,
               lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)) -> np.ndarray:
    """Randomly oriented thin rectangles (two triangles each), centres uniform in the box."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(np.asarray(lo, np.float64), np.asarray(hi, np.float64), (n_quads, 3))
    u = _uniform_sphere(rng, n_quads)
    v = _unit(np.cross(u, _uniform_sphere(rng, n_quads)))
    hu, hv = 0.5 * length * u, 0.5 * width * v
    p00, p10, p11, p01 = c - hu - hv, c + hu - hv, c + hu + hv, c - hu + hv
    tri = np.stack([np.stack([p00, p10, p11], 1), np.stack([p00, p11, p01], 1)], 1)
    return tri.reshape(-1, 3, 3).astype(np.float32)


def isotropic_tris(seed: int, n: int, edge: float = 0.01,
                   lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)) -> np.ndarray:
    """Near-equilateral triangles of edge ~``edge``, random orientation, centres uniform."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(np.asarray(lo, np.float64), np.asarray(hi, np.float64), (n, 3))
    nrm = _uniform_sphere(rng, n)
    e1, e2 = _perp_basis(nrm)
    rot = rng.uniform(0.0, 2 * math.pi, n)
    r = edge / math.sqrt(3.0)
    verts = []
    for j in range(3):
        ang = rot + 2 * math.pi * j / 3 + rng.normal(0.0, 0.05, n)
        rr = r * (1.0 + rng.normal(0.0, 0.05, n))
        verts.append(c + rr[:, None] * (np.cos(ang)[:, None] * e1 + np.sin(ang)[:, None] * e2))
    return np.stack(verts, 1).astype(np.float32)


# ----------------------------------------------------------------------------
# rays
# ----------------------------------------------------------------------------
def pinhole_rays(width: int, height: int, eye=(0.5, 0.5, 2.2), look=(0.5, 0.5, 0.5),
                 up=(0.0, 1.0, 0.0), vfov_deg: float = 40.0) -> np.ndarray:
    """Primary rays through pixel centres, row-major from the top-left pixel.

    Directions are normalised in float64 and then rounded; tmin = 0, tmax = +inf.
    """
    eye = np.asarray(eye, np.float64)
    fwd = _unit(np.asarray(look, np.float64) - eye)
    right = _unit(np.cross(fwd, np.asarray(up, np.float64)))
    upv = np.cross(right, fwd)
    th = math.tan(math.radians(vfov_deg) / 2)
    aspect = width / height
    j, i = np.meshgrid(np.arange(height, dtype=np.float64), np.arange(width, dtype=np.float64),
                       indexing="ij")
    px = ((i + 0.5) / width * 2.0 - 1.0) * th * aspect
    py = (1.0 - (j + 0.5) / height * 2.0) * th
    d = _unit(fwd + px[..., None] * right + py[..., None] * upv).reshape(-1, 3)
    rays = np.empty((d.shape[0], 8), np.float32)
    rays[:, 0:3] = eye
    rays[:, 3] = 0.0
    rays[:, 4:7] = d
    rays[:, 7] = np.inf
    return rays


def surface_bounce_rays(tris: np.ndarray, n: int, seed: int, offset: float = 2.0 ** -16) -> np.ndarray:
    """Diffuse secondary rays leaving the surface.

    Origin: a uniformly chosen triangle, a uniform point on it, pushed by
    ``offset`` along the normal of a randomly chosen side. Direction:
    cosine-weighted about that side's normal. tmin = 0, tmax = +inf.
    Degenerate (zero-area) triangles are skipped by resampling.
    """
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, tris.shape[0], n)
    v = tris[idx].astype(np.float64)  # [n, 3, 3] picked triangles only
    nrm = np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0])
    ln = np.linalg.norm(nrm, axis=-1)
    bad = ln == 0
    while bad.any():  # resample degenerate picks
        idx[bad] = rng.integers(0, tris.shape[0], int(bad.sum()))
        v[bad] = tris[idx[bad]].astype(np.float64)
        nrm = np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0])
        ln = np.linalg.norm(nrm, axis=-1)
        bad = ln == 0
    nrm = nrm / ln[:, None]
    side = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    nrm *= side[:, None]
    r1, r2 = rng.random(n), rng.random(n)
    su = np.sqrt(r1)
    b0, b1, b2 = 1.0 - su, su * (1.0 - r2), su * r2
    p = b0[:, None] * v[:, 0] + b1[:, None] * v[:, 1] + b2[:, None] * v[:, 2]
    e1, e2 = _perp_basis(nrm)
    r, phi = rng.random(n), rng.uniform(0.0, 2 * math.pi, n)
    sr = np.sqrt(r)
    d = (sr * np.cos(phi))[:, None] * e1 + (sr * np.sin(phi))[:, None] * e2 + \
        np.sqrt(np.maximum(0.0, 1.0 - r))[:, None] * nrm
    d = _unit(d)
    rays = np.empty((n, 8), np.float32)
    rays[:, 0:3] = p + offset * nrm
    rays[:, 3] = 0.0
    rays[:, 4:7] = d
    rays[:, 7] = np.inf
    return rays


def random_rays(n: int, seed: int, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)) -> np.ndarray:
    """Origins uniform in the box, directions uniform on the sphere."""
    rng = np.random.default_rng(seed)
    rays = np.empty((n, 8), np.float32)
    rays[:, 0:3] = rng.uniform(np.asarray(lo, np.float64), np.asarray(hi, np.float64), (n, 3))
    rays[:, 3] = 0.0
    rays[:, 4:7] = _uniform_sphere(rng, n)
    rays[:, 7] = np.inf
    return rays


# ----------------------------------------------------------------------------
# the named workloads
# ----------------------------------------------------------------------------
def scene_small(seed: int = 0) -> np.ndarray:
    """4,096 triangles: 128 curved strands x 32 segments, width 2e-3, unit cube."""
    return strands_random_walk(seed, 128, 32, 2e-3)


def rays_small(res: int = 256) -> np.ndarray:
    """res x res pinhole primary rays (65,536 at the default)."""
    return pinhole_rays(res, res)


def scene_hair_1m(seed: int = 1) -> np.ndarray:
    """1,000,002 triangles: 20k helical strands x 25 segments x 2 tris + ground plane."""
    s = strands_helical(seed, 20000, 25, 1e-3, 5e-3, 0.25,
                        (0.05, 0.0, 0.05), (0.95, 0.5, 0.95), axis=(0, 1, 0), max_tilt_deg=60.0)
    return np.concatenate([s, ground_plane(0.0)], 0)


def rays_hair_1m(tris: np.ndarray, seed: int = 1, width: int = 1920, height: int = 1080) -> np.ndarray:
    """1920x1080 primary rays followed by one diffuse surface ray per pixel."""
    prim = pinhole_rays(width, height)
    bounce = surface_bounce_rays(tris, prim.shape[0], seed + 10_000)
    return np.concatenate([prim, bounce], 0)


def scene_curly_12m(seed: int = 2, n_strands: int = 120_000) -> np.ndarray:
    """12M triangles: 120k curly strands x 50 segments x 2 tris, diagonal to the axes."""
    return strands_helical(seed, n_strands, 50, 5e-4, 3e-3, 0.3, (0.0, 0.0, 0.0),
                           (0.82, 0.82, 0.82), axis=(1, 1, 1), max_tilt_deg=15.0)


def rays_curly_12m(tris: np.ndarray, n: int = 8_000_000, seed: int = 2) -> np.ndarray:
    """Incoherent bounce rays leaving random points of the surface."""
    return surface_bounce_rays(tris, n, seed + 10_000)


def micro_scene(seed: int, n: int) -> np.ndarray:
    """A tiny random scene (1..64 tris) mixing the three triangle types."""
    rng = np.random.default_rng(seed)
    kind = seed % 3
    if kind == 0:
        t = strands_random_walk(seed, max(1, (n + 7) // 8), 8, 2e-3)
    elif kind == 1:
        t = thin_quads(seed, max(1, (n + 1) // 2), 0.2, 5e-3)
    else:
        t = isotropic_tris(seed, n, 0.2)
    t = t[:n]
    # place a few exactly on shared edges / axis-aligned to exercise ties
    if n >= 4 and rng.random() < 0.5:
        t[-1] = np.array([[0.25, 0.25, 0.5], [0.75, 0.25, 0.5], [0.25, 0.75, 0.5]], np.float32)
        t[-2] = np.array([[0.75, 0.25, 0.5], [0.75, 0.75, 0.5], [0.25, 0.75, 0.5]], np.float32)
    return t


def lattice_copies(kinds: int) -> np.ndarray:
    """Translated copies of `kinds` small random triangles on a 16 x 16 x 8 lattice of spacing 1/8:
    many child slots share one mask."""
    rng = np.random.default_rng(kinds)
    shapes = rng.uniform(0.0, 0.08, size=(kinds, 3, 3)).astype(np.float32)
    g = np.stack(np.meshgrid(np.arange(16), np.arange(16), np.arange(8), indexing="ij"), -1).reshape(-1, 3)
    tris = shapes[np.arange(g.shape[0]) % kinds] + (g.astype(np.float32) * np.float32(0.125))[:, None, :]
    return np.ascontiguousarray(tris, np.float32)


def segment_rows(seed: int) -> np.ndarray:
    """Zero-area triangles along x (3 to 12 per row) in 10 x 10 rows of constant (y, z): leaf boxes
    are line segments of surface area 0, so many distinct masks have importance 0."""
    rng = np.random.default_rng(seed)
    out = []
    for y in range(10):
        for z in range(10):
            n = int(rng.integers(3, 13))
            x0 = np.sort(rng.uniform(0, 1, n)).astype(np.float32)
            ln = rng.uniform(0.01, 0.1, n).astype(np.float32)
            for a, l in zip(x0, ln):
                v0 = np.array([a, y * 0.2, z * 0.2], np.float32)
                out.append([v0, v0 + np.array([l, 0, 0], np.float32), v0 + np.array([l * 0.5, 0, 0], np.float32)])
    return np.ascontiguousarray(np.array(out, np.float32))


@dataclass(frozen=True)
class BatchSpec:
    seed: int
    kind: str        # "strands" | "quads" | "iso"
    n_tris: int
    n_rays: int


def batch_specs(n_scenes: int = 64, seed0: int = 100, tri_lo: int = 10_000, tri_hi: int = 500_000,
                ray_lo: int = 16_000, ray_hi: int = 2_000_000) -> list:
    """Uneven scene/ray sizes, log-uniform, types cycling strands/quads/iso."""
    out = []
    kinds = ("strands", "quads", "iso")
    for i in range(n_scenes):
        rng = np.random.default_rng(seed0 + i)
        nt = int(round(math.exp(rng.uniform(math.log(tri_lo), math.log(tri_hi)))))
        nr = int(round(math.exp(rng.uniform(math.log(ray_lo), math.log(ray_hi)))))
        out.append(BatchSpec(seed0 + i, kinds[i % 3], nt, nr))
    return out


def batch_scene(spec: BatchSpec):
    """Triangles and rays (half primary, half random) for one batched scene."""
    if spec.kind == "strands":
        segs = 25
        ns = max(1, spec.n_tris // (2 * segs))
        t = strands_helical(spec.seed, ns, segs, 1e-3, 5e-3, 0.25, (0.05, 0.05, 0.05),
                            (0.95, 0.7, 0.95), axis=(0, 1, 0), max_tilt_deg=60.0)
    elif spec.kind == "quads":
        t = thin_quads(spec.seed, max(1, spec.n_tris // 2), 0.02, 5e-4)
    else:
        t = isotropic_tris(spec.seed, spec.n_tris, 0.01)
    t = t[:spec.n_tris]
    n_prim = spec.n_rays // 2
    res_w = max(1, int(math.sqrt(n_prim)))
    res_h = max(1, n_prim // res_w)
    prim = pinhole_rays(res_w, res_h)
    rnd = random_rays(spec.n_rays - prim.shape[0], spec.seed + 50_000)
    return t, np.concatenate([prim, rnd], 0)


# ----------------------------------------------------------------------------
# learned placement: training scenes and held-out scenes
# ----------------------------------------------------------------------------
@dataclass(frozen=True)
class PlacementSpec:
    seed: int
    kind: str        # "strands" | "curly" | "quads"
    n_tris: int
    n_rays: int


def placement_specs(n_scenes: int = 200, seed0: int = 5000, tri_lo: int = 100_000,
                    tri_hi: int = 2_000_000, n_rays: int = 262_144) -> list:
    """Training scenes: sizes log-uniform in [tri_lo, tri_hi], kinds cycling
    straight-ish strands / curly diagonal strands / thin quads."""
    kinds = ("strands", "curly", "quads")
    out = []
    for i in range(n_scenes):
        rng = np.random.default_rng(seed0 + i)
        nt = int(round(math.exp(rng.uniform(math.log(tri_lo), math.log(tri_hi)))))
        out.append(PlacementSpec(seed0 + i, kinds[i % 3], nt, n_rays))
    return out


def placement_scene(spec: PlacementSpec):
    """Triangles and rays (half pinhole primary, half surface bounce) of one scene."""
    rng = np.random.default_rng(spec.seed + 777)
    if spec.kind == "strands":
        segs = 25
        t = strands_helical(spec.seed, max(1, spec.n_tris // (2 * segs)), segs,
                            float(rng.uniform(5e-4, 2e-3)), float(rng.uniform(2e-3, 8e-3)),
                            float(rng.uniform(0.15, 0.35)), (0.05, 0.0, 0.05), (0.95, 0.5, 0.95),
                            axis=(0, 1, 0), max_tilt_deg=float(rng.uniform(20.0, 75.0)))
        t = np.concatenate([t[:max(0, spec.n_tris - 2)], ground_plane(0.0)], 0)
    elif spec.kind == "curly":
        segs = 50
        t = strands_helical(spec.seed, max(1, spec.n_tris // (2 * segs)), segs,
                            float(rng.uniform(3e-4, 1e-3)), float(rng.uniform(2e-3, 5e-3)),
                            float(rng.uniform(0.2, 0.4)), (0.0, 0.0, 0.0), (0.82, 0.82, 0.82),
                            axis=(1, 1, 1), max_tilt_deg=float(rng.uniform(5.0, 30.0)))
    else:
        t = thin_quads(spec.seed, max(1, spec.n_tris // 2), float(rng.uniform(0.01, 0.04)),
                       float(rng.uniform(2e-4, 1e-3)))
    t = np.ascontiguousarray(t[:spec.n_tris])
    n_prim = spec.n_rays // 2
    w = max(1, int(math.sqrt(n_prim)))
    prim = pinhole_rays(w, max(1, n_prim // w))
    bounce = surface_bounce_rays(t, spec.n_rays - prim.shape[0], spec.seed + 10_000)
    return t, np.concatenate([prim, bounce], 0)


def placement_heldout(k: int = 0, n_tris: int = 5_000_000, n_rays: int = 4_000_000):
    """Held-out scene k (seeds disjoint from the training range): a hair
    scene (k even) or a curly diagonal scene (k odd), with n_rays rays."""
    kind = "strands" if k % 2 == 0 else "curly"
    return placement_scene(PlacementSpec(90_000 + k, kind, n_tris, n_rays))
