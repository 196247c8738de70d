"""CPU oracle for subspace culling -- TEST INFRASTRUCTURE ONLY.

Plain, slow reference implementation of what the HIP path computes (BVH
build, ray-mask LUT, object masks, traversal with culling, codebook,
requirement LUTs and the mask search of Alg. 3, plus brute-force checks).
Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The product path never does, and the
oracle shares no code with the HIP library.

The arithmetic lives in ``sc_oracle.c`` (plain C, ``gcc -O2
-ffp-contract=off``); this module only builds it, loads it and marshals
numpy arrays. ``mlp.py`` holds the float64 reference of the placement MLP.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_SAN_LIB = os.path.join(_HERE, "liboracle_san.so")
_lib = None
# ORACLE_SANITIZE=1 builds and loads liboracle_san.so (AddressSanitizer + UBSan; run with gcc's
# libasan preloaded) instead
_SANITIZE = os.environ.get("ORACLE_SANITIZE") == "1"

MODES = {"none": 0, "raw": 1, "lut": 2, "sparse": 3}
FLAG_CULL = 1
FLAG_SHADOW = 2
LEAF_BIT = 0x80000000
EMPTY_REF = 0xFFFFFFFF
NO_HIT = 0xFFFFFFFF


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast math); sanitize=True builds the
    AddressSanitizer + UBSan variant liboracle_san.so."""
    out = _SAN_LIB if sanitize else _LIB
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        if sanitize:
            cmd[1:1] = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                        "-fno-omit-frame-pointer", "-g"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return out


def lib():
    global _lib
    if _lib is None:
        path = _SAN_LIB if _SANITIZE else _LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            build(force=True, sanitize=_SANITIZE)
        _lib = C.CDLL(path)
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def words_for(R: int) -> int:
    return (R * R * R + 63) // 64


@dataclass
class BVH:
    n_inner: int
    root: int
    depth: int
    cbox: np.ndarray   # float32 [n_inner, 12]: child0 lo, child0 hi, child1 lo, child1 hi
    cref: np.ndarray   # uint32 [n_inner, 2]
    range: np.ndarray  # uint32 [n_inner, 2]: first, count of the subtree
    perm: np.ndarray   # uint32 [n]: original triangle id at each leaf-order position

    def slot_boxes(self) -> np.ndarray:
        """[2*n_inner, 6] lo/hi of every child slot."""
        return self.cbox.reshape(-1, 6)


def leaf_slot_masks(masks: np.ndarray, bvh: "BVH", R: int) -> np.ndarray:
    """Masks kept only on the child slots whose child is a leaf: the slot of an
    inner child gets the full mask (all R^3 bits), which traversal never tests
    (a full mask always meets the ray mask). The same result as tracing with
    masks on leaf slots only."""
    W = words_for(R)
    out = np.array(masks, dtype=np.uint64, copy=True).reshape(-1, W)
    full = np.zeros(W, np.uint64)
    for w in range(W):
        bits = R ** 3 - 64 * w
        full[w] = np.uint64(0xFFFFFFFFFFFFFFFF) if bits >= 64 else np.uint64((1 << bits) - 1)
    inner = (bvh.cref.reshape(-1) & np.uint32(0x80000000)) == 0
    out[inner] = full
    return out.reshape(np.shape(masks))


def bvh_build(tris: np.ndarray, leaf_max: int = 4, bins: int = 32, depth_cap: int = 64) -> BVH:
    tris = np.ascontiguousarray(tris, np.float32)
    n = tris.shape[0]
    m = max(n, 1)
    cbox = np.zeros((m, 12), np.float32)
    cref = np.zeros((m, 2), np.uint32)
    rng = np.zeros((m, 2), np.uint32)
    perm = np.zeros(m, np.uint32)
    info = np.zeros(3, np.uint32)
    L = lib()
    L.orc_bvh_build.restype = C.c_int
    rc = L.orc_bvh_build(_p(tris), C.c_uint32(n), C.c_uint32(leaf_max), C.c_uint32(bins),
                         C.c_uint32(depth_cap), _p(cbox), _p(cref), _p(rng), _p(perm), _p(info))
    _check(rc, "bvh_build")
    ni = int(info[0])
    return BVH(ni, int(info[1]), int(info[2]), cbox[:ni].copy(), cref[:ni].copy(),
               rng[:ni].copy(), perm[:n].copy())


def raymask_lut(R: int) -> np.ndarray:
    W = words_for(R)
    out = np.zeros((R ** 6, W), np.uint64)
    _check(lib().orc_raymask_lut(C.c_uint32(R), _p(out)), "raymask_lut")
    return out


def default_bounds(tris: np.ndarray):
    """(origin_bound, delta) defaults: M = max |vertex coordinate|,
    origin_bound = 4 * max(1, M), delta = (max(1, M) + origin_bound) * 2^-16,
    all in float32."""
    M = np.float32(np.abs(tris).max()) if tris.size else np.float32(0)
    m1 = np.float32(max(np.float32(1.0), M))
    ob = np.float32(np.float32(4.0) * m1)
    delta = np.float32(np.float32(m1 + ob) * np.float32(2.0 ** -16))
    return float(ob), float(delta)


def object_masks(tris: np.ndarray, bvh: BVH, R: int, delta: float, nthreads: int = 0) -> np.ndarray:
    tris = np.ascontiguousarray(tris, np.float32)
    W = words_for(R)
    out = np.zeros((max(2 * bvh.n_inner, 1), W), np.uint64)
    L = lib()
    rc = L.orc_object_masks(_p(tris), _p(bvh.perm), C.c_uint32(bvh.n_inner), _p(bvh.cbox),
                            _p(bvh.cref), _p(bvh.range), C.c_uint32(R), C.c_float(delta),
                            _p(out), C.c_int(nthreads))
    _check(rc, "object_masks")
    return out[:2 * bvh.n_inner]


def fill_table(R: int) -> np.ndarray:
    """Filling-pattern table of Alg. 2: [R^6, W], key ((((x0*R+y0)*R+z0)*R+x1)*R+y1)*R+z1."""
    out = np.zeros((R ** 6, words_for(R)), np.uint64)
    _check(lib().orc_fill_table(C.c_uint32(R), _p(out)), "fill_table")
    return out


def fill_one(parent_box, child_mask, child_box, R: int, delta: float, table=None) -> np.ndarray:
    """Alg. 2 for one child mask: the parent voxels its set voxels fill."""
    table = fill_table(R) if table is None else table
    pb = np.ascontiguousarray(parent_box, np.float32)
    cb = np.ascontiguousarray(child_box, np.float32)
    cm = np.ascontiguousarray(child_mask, np.uint64)
    out = np.zeros(words_for(R), np.uint64)
    _check(lib().orc_fill_one(_p(pb[:3].copy()), _p(pb[3:].copy()), _p(cm), _p(cb[:3].copy()), _p(cb[3:].copy()),
                              C.c_uint32(R), C.c_float(delta), _p(table), _p(out)), "fill_one")
    return out


def approx_masks(tris: np.ndarray, bvh: BVH, R: int, delta: float, L: int, table=None) -> np.ndarray:
    """Child-slot masks with the approximation of Sect. 3.2.1 / Alg. 2 at level L."""
    tris = np.ascontiguousarray(tris, np.float32)
    table = fill_table(R) if table is None else np.ascontiguousarray(table, np.uint64)
    out = np.zeros((max(2 * bvh.n_inner, 1), words_for(R)), np.uint64)
    _check(lib().orc_approx_masks(_p(tris), _p(bvh.perm), C.c_uint32(bvh.n_inner), _p(bvh.cbox), _p(bvh.cref),
                                  _p(bvh.range), C.c_uint32(R), C.c_float(delta), C.c_uint32(L), _p(table),
                                  _p(out)), "approx_masks")
    return out[:2 * bvh.n_inner]


@dataclass
class Hits:
    prim: np.ndarray        # uint32, NO_HIT on a miss
    t: np.ndarray           # float32, +inf on a miss
    box_tests: np.ndarray
    tri_tests: np.ndarray
    mask_tests: np.ndarray
    mask_culls: np.ndarray
    slot_fp: np.ndarray | None = None
    deepest: np.ndarray | None = None  # trace4(stack_depth=True): stack entries beneath the visited node
    cb_refs: np.ndarray | None = None  # trace4(codebook_refs=True), LUT mode: mask tests per codebook entry


RAY_MASKS = {"lut": 0, "lut2r": 1, "ideal": 2}


def raymask_lut2(R: int) -> np.ndarray:
    """Ray-mask table at ray resolution 2R: [(2R)^6, W] R-grid masks."""
    F = 2 * R
    out = np.zeros((F ** 6, words_for(R)), np.uint64)
    _check(lib().orc_raymask_lut2(C.c_uint32(R), _p(out)), "raymask_lut2")
    return out


def ideal_mask(box, o, d, t0, t1, R):
    """Ideal ray mask of segment o + t d, t in [t0, t1], in box (lo xyz, hi xyz)."""
    b = np.ascontiguousarray(box, np.float32)
    out = np.zeros(words_for(R), np.uint64)
    _check(lib().orc_ideal_mask(_p(b[:3].copy()), _p(b[3:].copy()), _p(np.asarray(o, np.float32)),
                                _p(np.asarray(d, np.float32)), C.c_float(t0), C.c_float(t1), C.c_uint32(R),
                                _p(out)), "ideal_mask")
    return out


def trace(tris, bvh: BVH, rays, *, mode="none", R=6, masks=None, codebook=None, cidx=None,
          placed=None, lut=None, origin_bound=None, cull=True, shadow=False, nthreads=0,
          ray_masks="lut", lut2=None, test_max=0) -> Hits:
    """Traversal with culling. mode "raw": masks per slot; "lut": codebook +
    cidx; "sparse": masks per slot used only where placed[slot] != 0. A slot
    whose mask has more than test_max set bits is never tested (0 = R^3 - 1:
    only a full mask). ray_masks: "lut" (the table at R, the method), "lut2r"
    (the table at 2R) or "ideal" (every voxel the segment crosses), the last
    two as tightness references."""
    tris = np.ascontiguousarray(tris, np.float32)
    rays = np.ascontiguousarray(rays, np.float32)
    n = rays.shape[0]
    if origin_bound is None:
        origin_bound = default_bounds(tris)[0]
    mcode = MODES[mode]
    if mcode and lut is None:
        lut = raymask_lut(R)
    hits = np.zeros((max(n, 1), 4), np.uint32)
    extra = np.zeros((max(n, 1), 2), np.uint32)
    fp = np.zeros(max(2 * bvh.n_inner, 1), np.uint32) if shadow else None
    flags = (FLAG_CULL if cull else 0) | (FLAG_SHADOW if shadow else 0)
    masks = None if masks is None else np.ascontiguousarray(masks, np.uint64)
    codebook = None if codebook is None else np.ascontiguousarray(codebook, np.uint64)
    cidx = None if cidx is None else np.ascontiguousarray(cidx, np.uint16)
    placed = None if placed is None else np.ascontiguousarray(placed, np.uint8)
    kind = RAY_MASKS[ray_masks]
    if kind == 1 and lut2 is None:
        lut2 = raymask_lut2(R)
    rc = lib().orc_trace_ex(_p(tris), _p(bvh.perm), _p(bvh.cbox), _p(bvh.cref), C.c_uint32(bvh.root),
                            C.c_uint32(bvh.depth), C.c_uint32(R), C.c_uint32(mcode), _p(masks),
                            _p(codebook), _p(cidx), _p(placed), _p(lut), C.c_float(origin_bound),
                            C.c_uint32(flags), _p(rays), C.c_uint32(n), _p(hits), _p(extra), _p(fp),
                            C.c_int(nthreads), C.c_uint32(kind), _p(lut2), C.c_uint32(test_max))
    _check(rc, "trace")
    hits, extra = hits[:n], extra[:n]
    return Hits(hits[:, 0].copy(), hits[:, 1].view(np.float32).copy(), hits[:, 2].copy(),
                hits[:, 3].copy(), extra[:, 0].copy(), extra[:, 1].copy(),
                None if fp is None else fp[:2 * bvh.n_inner])


@dataclass
class BVH4:
    """4-wide BVH collapsed from a binary one: child c of node m has box
    box4[m, c] (lo xyz, hi xyz), ref ref4[m, c] (leaf refs as in the binary
    BVH, inner refs = 4-wide node index, EMPTY for an unused slot) and comes
    from binary child slot src4[m, c] (EMPTY when unused)."""
    box4: np.ndarray   # float32 [n4, 4, 6]
    ref4: np.ndarray   # uint32 [n4, 4]
    src4: np.ndarray   # uint32 [n4, 4]
    root: int
    depth: int         # of the binary BVH it came from (bounds the 4-wide depth)

    @property
    def n4(self) -> int:
        return self.ref4.shape[0]


def bvh4_collapse(bvh: BVH) -> BVH4:
    m = max(bvh.n_inner, 1)
    box4 = np.zeros((m, 4, 6), np.float32)
    ref4 = np.zeros((m, 4), np.uint32)
    src4 = np.zeros((m, 4), np.uint32)
    n4, root4 = C.c_uint32(0), C.c_uint32(0)
    _check(lib().orc_bvh4_collapse(_p(bvh.cbox), _p(bvh.cref), C.c_uint32(bvh.n_inner), C.c_uint32(bvh.root),
                                   _p(box4), _p(ref4), _p(src4), C.byref(n4), C.byref(root4)), "bvh4_collapse")
    k = n4.value
    return BVH4(box4[:k].copy(), ref4[:k].copy(), src4[:k].copy(), root4.value, bvh.depth)


@dataclass
class Quant4:
    """Quantised child boxes of a 4-wide BVH (orc_quantise4): per node the
    minimum corner lo [n4, 3] of its used children, the biased exponents
    ebias [n4, 3] (scale 2^(ebias - 127) per axis), the 8-bit planes
    q [n4, 4, 6] (qlo xyz, qhi xyz per child) and the decoded boxes
    dec [n4, 4, 6], laid out as BVH4.box4."""
    lo: np.ndarray
    ebias: np.ndarray
    q: np.ndarray
    dec: np.ndarray


def quantise4(bvh4: BVH4) -> Quant4:
    """Child boxes of every 4-wide node as 8-bit offsets from the node's minimum
    corner in steps of a power of two per axis, rounded outward (the child-box
    compression of compressed wide BVHs; not part of the paper)."""
    m = max(bvh4.n4, 1)
    lo = np.zeros((m, 3), np.float32)
    eb = np.zeros((m, 3), np.uint8)
    q = np.zeros((m, 4, 6), np.uint8)
    dec = np.zeros((m, 4, 6), np.float32)
    if bvh4.n4:
        _check(lib().orc_quantise4(_p(np.ascontiguousarray(bvh4.box4, np.float32)),
                                   _p(np.ascontiguousarray(bvh4.ref4, np.uint32)), C.c_uint32(bvh4.n4),
                                   _p(lo), _p(eb), _p(q), _p(dec)), "quantise4")
    k = bvh4.n4
    return Quant4(lo[:k].copy(), eb[:k].copy(), q[:k].copy(), dec[:k].copy())


def decoded_bvh4(bvh4: BVH4, qt: Quant4) -> BVH4:
    """The 4-wide BVH with every child box replaced by its decoded box."""
    return BVH4(qt.dec.copy(), bvh4.ref4.copy(), bvh4.src4.copy(), bvh4.root, bvh4.depth)


def with_slot_boxes(bvh: BVH, bvh4: BVH4) -> BVH:
    """A copy of the binary BVH whose child slots that a 4-wide node uses carry
    that node's box for the child (the decoded box, for a decoded BVH4); masks,
    approximate masks and codebook importances built on it then belong to the
    boxes the 4-wide traversal tests. Slots no 4-wide node uses keep theirs."""
    cbox = bvh.cbox.copy().reshape(-1, 6)
    used = bvh4.ref4 != EMPTY_REF
    cbox[bvh4.src4[used]] = bvh4.box4[used]
    return BVH(bvh.n_inner, bvh.root, bvh.depth, cbox.reshape(bvh.cbox.shape), bvh.cref.copy(),
               bvh.range.copy(), bvh.perm.copy())


def trace4(tris, bvh: BVH, bvh4: BVH4, rays, *, mode="none", R=6, masks=None, codebook=None, cidx=None,
           placed=None, lut=None, origin_bound=None, cull=True, shadow=False, nthreads=0,
           stack_depth=False, test_max=0, codebook_refs=False) -> Hits:
    """Alg. 4 on the 4-wide BVH; masks, codebook indices, shadow counts and
    test_max are as for trace(). stack_depth=True also returns, per ray, the
    most stack entries held beneath the node being visited (Hits.deepest);
    codebook_refs=True (LUT mode) the number of mask tests that read each
    codebook entry (Hits.cb_refs)."""
    tris = np.ascontiguousarray(tris, np.float32)
    rays = np.ascontiguousarray(rays, np.float32)
    n = rays.shape[0]
    if origin_bound is None:
        origin_bound = default_bounds(tris)[0]
    mcode = MODES[mode]
    if mcode and lut is None:
        lut = raymask_lut(R)
    hits = np.zeros((max(n, 1), 4), np.uint32)
    extra = np.zeros((max(n, 1), 2), np.uint32)
    fp = np.zeros(max(2 * bvh.n_inner, 1), np.uint32) if shadow else None
    flags = (FLAG_CULL if cull else 0) | (FLAG_SHADOW if shadow else 0)
    masks = None if masks is None else np.ascontiguousarray(masks, np.uint64)
    codebook = None if codebook is None else np.ascontiguousarray(codebook, np.uint64)
    cidx = None if cidx is None else np.ascontiguousarray(cidx, np.uint16)
    placed = None if placed is None else np.ascontiguousarray(placed, np.uint8)
    b4 = np.ascontiguousarray(bvh4.box4) if bvh4.n4 else np.zeros((1, 4, 6), np.float32)
    r4 = np.ascontiguousarray(bvh4.ref4) if bvh4.n4 else np.zeros((1, 4), np.uint32)
    s4 = np.ascontiguousarray(bvh4.src4) if bvh4.n4 else np.zeros((1, 4), np.uint32)
    deep = np.zeros(max(n, 1), np.uint32) if stack_depth else None
    refs = np.zeros(max(codebook.shape[0], 1), np.uint32) if (codebook_refs and mode == "lut") else None
    rc = lib().orc_trace4(_p(tris), _p(bvh.perm), _p(b4), _p(r4), _p(s4), C.c_uint32(bvh4.root),
                          C.c_uint32(bvh4.depth), C.c_uint32(R), C.c_uint32(mcode), _p(masks), _p(codebook),
                          _p(cidx), _p(placed), _p(lut), C.c_float(origin_bound), C.c_uint32(flags), _p(rays),
                          C.c_uint32(n), _p(hits), _p(extra), _p(fp), C.c_int(nthreads), _p(deep),
                          C.c_uint32(test_max), _p(refs))
    _check(rc, "trace4")
    hits, extra = hits[:n], extra[:n]
    return Hits(hits[:, 0].copy(), hits[:, 1].view(np.float32).copy(), hits[:, 2].copy(),
                hits[:, 3].copy(), extra[:, 0].copy(), extra[:, 1].copy(),
                None if fp is None else fp[:2 * bvh.n_inner], None if deep is None else deep[:n],
                None if refs is None else refs[:codebook.shape[0]])


def bit_table(R: int, cb, lut=None) -> np.ndarray:
    """2-D bit table: uint32 [R^6, K/32], bit k of row key = (LUT[key] AND cb[k]) != 0."""
    cb = np.ascontiguousarray(cb, np.uint64)
    K = cb.shape[0]
    lut = raymask_lut(R) if lut is None else np.ascontiguousarray(lut, np.uint64)
    out = np.zeros((R ** 6, K // 32), np.uint32)
    _check(lib().orc_bit_table(_p(lut), C.c_uint32(R), _p(cb), C.c_uint32(K), _p(out)), "bit_table")
    return out


def brute_closest(tris, rays, nthreads=0):
    tris = np.ascontiguousarray(tris, np.float32)
    rays = np.ascontiguousarray(rays, np.float32)
    n = rays.shape[0]
    out = np.zeros((max(n, 1), 2), np.uint32)
    _check(lib().orc_brute_closest(_p(tris), C.c_uint32(tris.shape[0]), _p(rays), C.c_uint32(n),
                                   _p(out), C.c_int(nthreads)), "brute_closest")
    return out[:n, 0].copy(), out[:n, 1].view(np.float32).copy()


def codebook(masks, slot_boxes, R, K):
    masks = np.ascontiguousarray(masks, np.uint64)
    boxes = np.ascontiguousarray(slot_boxes, np.float32)
    cb = np.zeros((K, words_for(R)), np.uint64)
    _check(lib().orc_codebook(_p(masks), _p(boxes), C.c_uint32(masks.shape[0]), C.c_uint32(R),
                              C.c_uint32(K), _p(cb)), "codebook")
    return cb


def req_luts(cb, R):
    K = cb.shape[0]
    nch = (R ** 3 + 7) // 8
    req = np.zeros((nch, 256, K // 64), np.uint64)
    _check(lib().orc_req_luts(_p(np.ascontiguousarray(cb, np.uint64)), C.c_uint32(K),
                              C.c_uint32(R), _p(req)), "req_luts")
    return req


def alg3(masks, req, K, R):
    masks = np.ascontiguousarray(masks, np.uint64)
    out = np.zeros(max(masks.shape[0], 1), np.uint16)
    _check(lib().orc_alg3(_p(masks), C.c_uint32(masks.shape[0]), _p(req), C.c_uint32(K),
                          C.c_uint32(R), _p(out)), "alg3")
    return out[:masks.shape[0]]


def naive_search(masks, cb, R):
    masks = np.ascontiguousarray(masks, np.uint64)
    out = np.zeros(max(masks.shape[0], 1), np.uint16)
    _check(lib().orc_naive_search(_p(masks), C.c_uint32(masks.shape[0]),
                                  _p(np.ascontiguousarray(cb, np.uint64)), C.c_uint32(cb.shape[0]),
                                  C.c_uint32(R), _p(out)), "naive_search")
    return out[:masks.shape[0]]


def compress(masks, slot_boxes, R, K):
    """Codebook + indices the way the compressed node layout stores them."""
    cb = codebook(masks, slot_boxes, R, K)
    req = req_luts(cb, R)
    return cb, alg3(masks, req, K, R)


def voxelize_tri(tri, lo, hi, R, delta):
    """Mask bits of one triangle in the box (lo, hi) -> uint64 [W]."""
    out = np.zeros(words_for(R), np.uint64)
    _check(lib().orc_voxelize_tri(_p(np.ascontiguousarray(tri, np.float32)),
                                  _p(np.ascontiguousarray(lo, np.float32)),
                                  _p(np.ascontiguousarray(hi, np.float32)), C.c_uint32(R),
                                  C.c_float(delta), _p(out)), "voxelize_tri")
    return out


def mask_bits(m, R) -> np.ndarray:
    """uint64 [..., W] -> bool [..., R^3] (bit x + R*y + R^2*z)."""
    m = np.asarray(m, np.uint64)
    bits = ((m[..., :, None] >> np.arange(64, dtype=np.uint64)) & np.uint64(1)).astype(bool)
    return bits.reshape(*m.shape[:-1], -1)[..., :R ** 3]


def ray_mask(lo, hi, o, d, t0, t1, R, lut):
    """Alg. 1 for one box and segment -> uint64 [W]."""
    out = np.zeros(words_for(R), np.uint64)
    f = lambda a: np.ascontiguousarray(a, np.float32)
    _check(lib().orc_ray_mask(_p(f(lo)), _p(f(hi)), _p(f(o)), _p(f(d)), C.c_float(t0),
                              C.c_float(t1), C.c_uint32(R), _p(lut), _p(out)), "ray_mask")
    return out


def slot_masks(tris, bvh: BVH, slots, R, delta, nthreads=0):
    """Object masks of the given child slots only -> uint64 [len(slots), W]."""
    slots = np.ascontiguousarray(slots, np.uint32)
    out = np.zeros((max(slots.size, 1), words_for(R)), np.uint64)
    _check(lib().orc_slot_masks(_p(np.ascontiguousarray(tris, np.float32)), _p(bvh.perm), _p(bvh.cbox),
                                _p(bvh.cref), _p(bvh.range), _p(slots), C.c_uint32(slots.size),
                                C.c_uint32(R), C.c_float(delta), _p(out), C.c_int(nthreads)), "slot_masks")
    return out[:slots.size]


def cpu_threads() -> int:
    import os as _os
    return len(_os.sched_getaffinity(0))
