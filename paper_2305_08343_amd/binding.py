"""Python binding of libsubcull (ctypes; argument marshalling only).

Every computation runs in the HIP library; torch supplies device memory and
streams. The names follow the C ABI in ``include/subcull.h``. Importing this
module on a machine without the built library raises immediately -- there
is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# SUBCULL_LIB may name another build of the same library (e.g. libsubcull_san.so, host code
# under AddressSanitizer); there is no fallback of any kind
LIB_PATH = os.environ.get("SUBCULL_LIB") or os.path.join(_HERE, "libsubcull.so")

SC_OK = 0
SC_MASK_NONE, SC_MASK_RAW, SC_MASK_LUT, SC_MASK_SPARSE = 0, 1, 2, 3
SC_TRACE_CULL, SC_TRACE_SHADOW, SC_TRACE_SORT = 1, 2, 4
MODES = {"none": SC_MASK_NONE, "raw": SC_MASK_RAW, "lut": SC_MASK_LUT, "sparse": SC_MASK_SPARSE}
NO_HIT = 0xFFFFFFFF


class SubcullError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {detail} (status {status})")
        self.status = status


class sc_allocator(C.Structure):
    _fields_ = [("alloc", C.c_void_p), ("free", C.c_void_p), ("user", C.c_void_p)]


class sc_build_params(C.Structure):
    _fields_ = [("R", C.c_uint32), ("leaf_max", C.c_uint32), ("sah_bins", C.c_uint32),
                ("depth_cap", C.c_uint32), ("mode", C.c_uint32), ("codebook_size", C.c_uint32),
                ("delta", C.c_float), ("origin_bound", C.c_float),
                ("mask_placement", C.c_void_p), ("placement_len", C.c_uint32), ("width", C.c_uint32),
                ("approx_levels", C.c_uint32), ("bit_table", C.c_uint32), ("mask_slots", C.c_uint32),
                ("quantise", C.c_uint32), ("mask_test_max", C.c_uint32)]


class sc_scene_info(C.Structure):
    _fields_ = [("n_tris", C.c_uint32), ("n_inner", C.c_uint32), ("depth", C.c_uint32),
                ("root_ref", C.c_uint32), ("R", C.c_uint32), ("mode", C.c_uint32),
                ("codebook_size", C.c_uint32), ("words", C.c_uint32), ("node_bytes", C.c_uint32),
                ("n_masked", C.c_uint32), ("width", C.c_uint32), ("n_nodes", C.c_uint32),
                ("approx_levels", C.c_uint32), ("bit_table", C.c_uint32), ("mask_test_max", C.c_uint32),
                ("delta", C.c_float), ("origin_bound", C.c_float),
                ("device_bytes", C.c_uint64), ("ms_bvh", C.c_double), ("ms_masks", C.c_double),
                ("ms_codebook", C.c_double), ("ms_compress", C.c_double)]


class sc_tune(C.Structure):
    _fields_ = [("block", C.c_uint32), ("stack", C.c_uint32), ("chunk", C.c_uint32),
                ("parts", C.c_uint32), ("waves", C.c_uint32), ("sort", C.c_uint32), ("codebook", C.c_uint32),
                ("gather", C.c_uint32), ("refill", C.c_uint32)]


class sc_batch_item(C.Structure):
    _fields_ = [("scene", C.c_void_p), ("d_rays", C.c_void_p), ("n", C.c_uint32), ("d_hits", C.c_void_p),
                ("d_extra", C.c_void_p), ("d_slot_fp", C.c_void_p)]


class sc_scene_host(C.Structure):
    _fields_ = [("cbox", C.c_void_p), ("cref", C.c_void_p), ("range", C.c_void_p),
                ("perm", C.c_void_p), ("masks", C.c_void_p), ("codebook", C.c_void_p),
                ("cidx", C.c_void_p)]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)

# Every symbol the header declares, with its ctypes signature.
_SIGS = {
    "sc_build_params_default": (None, [C.POINTER(sc_build_params)]),
    "sc_create": (C.c_int, [C.c_int, C.POINTER(sc_allocator), C.POINTER(C.c_void_p)]),
    "sc_destroy": (C.c_int, [C.c_void_p]),
    "sc_scene_build": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.POINTER(sc_build_params),
                                 C.c_void_p, C.POINTER(C.c_void_p)]),
    "sc_scene_destroy": (C.c_int, [C.c_void_p]),
    "sc_bvh_build_host": (C.c_int, [C.c_void_p, C.c_uint32, C.POINTER(sc_build_params),
                                    C.POINTER(sc_scene_host), C.POINTER(sc_scene_info)]),
    "sc_scene_get_info": (C.c_int, [C.c_void_p, C.POINTER(sc_scene_info)]),
    "sc_scene_export": (C.c_int, [C.c_void_p, C.POINTER(sc_scene_host)]),
    "sc_trace": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_uint32, C.c_void_p, C.c_void_p,
                           C.c_void_p, C.c_void_p]),
    "sc_trace_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_uint32, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p]),
    "sc_scene_export4": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sc_scene_export_bit_table": (C.c_int, [C.c_void_p, C.c_void_p]),
    "sc_ray_order": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p]),
    "sc_trace_batch": (C.c_int, [C.c_void_p, C.POINTER(sc_batch_item), C.c_uint32, C.c_uint32, C.c_void_p]),
    "sc_batch_create": (C.c_int, [C.c_void_p, C.POINTER(sc_batch_item), C.c_uint32, C.c_uint32,
                                  C.POINTER(C.c_void_p)]),
    "sc_batch_launch": (C.c_int, [C.c_void_p, C.c_void_p]),
    "sc_batch_destroy": (C.c_int, [C.c_void_p]),
    "sc_set_tune": (C.c_int, [C.c_void_p, C.POINTER(sc_tune)]),
    "sc_get_tune": (C.c_int, [C.c_void_p, C.POINTER(sc_tune)]),
    "sc_set_device_checks": (C.c_int, [C.c_void_p, C.c_int]),
    "sc_get_check_flags": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint32), C.c_int]),
    "sc_set_check_limits": (C.c_int, [C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32]),
    "sc_raymask_lut": (C.c_int, [C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p]),
    "sc_compress_masks": (C.c_int, [C.c_void_p, C.c_uint32, C.c_void_p, C.c_uint32, C.c_void_p,
                                    C.c_uint32, C.c_void_p, C.c_void_p]),
    "sc_slot_features": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "sc_mlp_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p,
                                 C.c_void_p]),
    "sc_mlp_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sc_mlp_adam": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32,
                              C.c_float, C.c_float, C.c_float, C.c_float, C.c_void_p]),
    "sc_place_top": (C.c_int, [C.c_void_p, C.c_uint32, C.c_uint32, C.c_void_p]),
    "sc_status_string": (C.c_char_p, [C.c_int]),
    "sc_last_error": (C.c_char_p, []),
}

_lib = None


def load():
    """Load libsubcull.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2305_08343_amd.build` (ROCm hipcc, gfx950)")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(status: int, where: str):
    if status != SC_OK:
        lib = load()
        raise SubcullError(status, where, lib.sc_last_error().decode() or
                           lib.sc_status_string(status).decode())


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _on_stream(stream):
    """Context in which a call's input copies and output allocations are made on `stream`, the
    stream the library runs the call on. A stream other than the current one first waits for the
    current stream, so inputs produced there are complete before the library reads them, and
    temporaries allocated under it belong to it in torch's caching allocator."""
    import contextlib

    import torch
    if stream is None:
        return contextlib.nullcontext()
    cur = torch.cuda.current_stream(stream.device)
    if stream != cur:
        stream.wait_stream(cur)
    return torch.cuda.stream(stream)


SC_CHECK_NODE, SC_CHECK_TRI, SC_CHECK_STACK, SC_CHECK_INDEX = 1, 2, 4, 8
SC_MLP_PARAMS, SC_MLP_GRAD_PARTS = 5057, 32


def mlp_work_floats(n: int) -> int:
    """Floats of the scratch sc_mlp_backward needs for a batch of n (SC_MLP_WORK_FLOATS)."""
    return n * 130 + SC_MLP_GRAD_PARTS * SC_MLP_PARAMS
# (device, bits) of every context closed with device checks on and a failed check not reset
CHECK_FAILURES = []


class Context:
    """An sc_ctx on one device; scene memory comes from torch's allocator.

    ``checks=True`` (or the environment variable SUBCULL_DEBUG=1 when ``checks`` is None) runs
    the traversal kernels with device checks; ``check_flags()`` reads what failed.
    ``allocator=(alloc, free)`` routes the library's device memory through two callables instead:
    ``alloc(nbytes, stream) -> int`` (a device address usable on the stream handle, or 0 when the
    memory cannot be had) and ``free(ptr, nbytes, stream)``."""

    def __init__(self, device: int = 0, torch_memory: bool = True, checks=None, allocator=None):
        import torch
        lib = load()
        self.device = device
        self._keep = []
        alloc_p = None
        if allocator is not None:
            user_alloc, user_free = allocator

            def _alloc(nbytes, stream, user):
                try:
                    return user_alloc(int(nbytes), stream or 0) or None
                except Exception:
                    return None

            def _free(ptr, nbytes, stream, user):
                user_free(ptr, int(nbytes), stream or 0)

            fa, ff = _ALLOC_FN(_alloc), _FREE_FN(_free)
            self._keep += [fa, ff]
            self._alloc = sc_allocator(C.cast(fa, C.c_void_p), C.cast(ff, C.c_void_p), None)
            alloc_p = C.byref(self._alloc)
        elif torch_memory:
            def _alloc(nbytes, stream, user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), device, stream or 0)
                except Exception:
                    return None

            def _free(ptr, nbytes, stream, user):
                torch.cuda.caching_allocator_delete(ptr)

            fa, ff = _ALLOC_FN(_alloc), _FREE_FN(_free)
            self._keep += [fa, ff]
            self._alloc = sc_allocator(C.cast(fa, C.c_void_p), C.cast(ff, C.c_void_p), None)
            alloc_p = C.byref(self._alloc)
        h = C.c_void_p()
        torch.cuda.set_device(device)
        _check(lib.sc_create(device, alloc_p, C.byref(h)), "sc_create")
        self.handle = h
        if checks is None:
            checks = os.environ.get("SUBCULL_DEBUG") == "1"
        if checks:
            try:
                _check(lib.sc_set_device_checks(self.handle, 1), "sc_set_device_checks")
            except SubcullError:
                lib.sc_destroy(self.handle)  # a context that failed to start holds nothing
                self.handle = None
                raise
        self.checks = bool(checks)

    def set_device_checks(self, on: bool):
        _check(load().sc_set_device_checks(self.handle, 1 if on else 0), "sc_set_device_checks")
        self.checks = bool(on)

    def check_flags(self, reset: bool = False) -> int:
        """OR of the SC_CHECK_* bits of every failed device check since the last reset."""
        v = C.c_uint32(0)
        _check(load().sc_get_check_flags(self.handle, C.byref(v), 1 if reset else 0), "sc_get_check_flags")
        return int(v.value)

    def set_check_limits(self, stack: int = 0, nodes: int = 0, tris: int = 0):
        """Lower the checked limits below the scene's own (0 = the scene's value)."""
        _check(load().sc_set_check_limits(self.handle, stack, nodes, tris), "sc_set_check_limits")

    def close(self):
        if getattr(self, "handle", None):
            if getattr(self, "checks", False):
                try:
                    bits = self.check_flags()
                except SubcullError:
                    bits = 0  # the device is in error; the destroy below still runs
                if bits:
                    CHECK_FAILURES.append((self.device, bits))
            load().sc_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tune(self, block: int = 256, stack: int = 8, chunk: int = 1, parts: int = 8, waves: int = 0,
                 sort: int = 0, codebook: int = 0, gather: int = 16, refill: int = 16):
        """Traversal launch shape for later traces (results never depend on it)."""
        _check(load().sc_set_tune(self.handle, C.byref(sc_tune(block, stack, chunk, parts, waves, sort,
                                                               codebook, gather, refill))), "sc_set_tune")

    def get_tune(self) -> dict:
        t = sc_tune()
        _check(load().sc_get_tune(self.handle, C.byref(t)), "sc_get_tune")
        return {"block": t.block, "stack": t.stack, "chunk": t.chunk, "parts": t.parts, "waves": t.waves,
                "sort": t.sort, "codebook": t.codebook, "gather": t.gather, "refill": t.refill}

    # ---- placement MLP (device tensors in, device tensors out)
    def mlp_forward(self, params, x, act=None, stream=None):
        import torch
        n = x.shape[0]
        y = torch.empty(max(n, 1), dtype=torch.float32, device=x.device)
        _check(load().sc_mlp_forward(self.handle, _ptr(params), _ptr(x), n, _ptr(y), _ptr(act),
                                     _stream_ptr(stream)), "sc_mlp_forward")
        return y[:n]

    def mlp_backward(self, params, x, act, y, t, grad, work, loss=None, stream=None):
        _check(load().sc_mlp_backward(self.handle, _ptr(params), _ptr(x), _ptr(act), _ptr(y), _ptr(t),
                                      x.shape[0], _ptr(grad), _ptr(work), _ptr(loss), _stream_ptr(stream)),
               "sc_mlp_backward")

    def mlp_adam(self, params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _check(load().sc_mlp_adam(self.handle, _ptr(params), _ptr(grad), _ptr(m), _ptr(v), step, lr, beta1,
                                  beta2, eps, _stream_ptr(stream)), "sc_mlp_adam")

    def raymask_lut(self, R: int, stream=None):
        """Device ray-mask LUT as uint64 numpy array [R^6, W] (copies back)."""
        import torch
        W = (R ** 3 + 63) // 64
        out = torch.empty((R ** 6, W), dtype=torch.int64, device=f"cuda:{self.device}")
        _check(load().sc_raymask_lut(self.handle, R, _ptr(out), _stream_ptr(stream)), "sc_raymask_lut")
        torch.cuda.synchronize(self.device)
        return out.cpu().numpy().view(np.uint64)

    def compress_masks(self, R: int, codebook: np.ndarray, masks: np.ndarray, stream=None):
        """Alg. 3 on the device for given masks and codebook -> uint16 indices."""
        import torch
        dev = f"cuda:{self.device}"
        cb = torch.from_numpy(np.ascontiguousarray(codebook, np.uint64).view(np.int64)).to(dev)
        m = torch.from_numpy(np.ascontiguousarray(masks, np.uint64).view(np.int64)).to(dev)
        n = masks.shape[0]
        idx = torch.empty(max(n, 1), dtype=torch.int16, device=dev)
        _check(load().sc_compress_masks(self.handle, R, _ptr(cb), codebook.shape[0], _ptr(m), n,
                                        _ptr(idx), _stream_ptr(stream)), "sc_compress_masks")
        return idx[:n].cpu().numpy().view(np.uint16)


def bvh_build_host(tris, leaf_max: int = 4, bins: int = 32, depth_cap: int = 64) -> dict:
    """The library's host BVH builder alone (no device): cbox, cref, range, perm, depth, root."""
    lib = load()
    tris = np.ascontiguousarray(tris, np.float32)
    n = tris.shape[0]
    m = max(n, 1)
    out = {"cbox": np.zeros((m, 12), np.float32), "cref": np.zeros((m, 2), np.uint32),
           "range": np.zeros((m, 2), np.uint32), "perm": np.zeros(m, np.uint32)}
    hs = sc_scene_host(*(out[k].ctypes.data_as(C.c_void_p) for k in ("cbox", "cref", "range", "perm")),
                       None, None, None)
    p = sc_build_params()
    lib.sc_build_params_default(C.byref(p))
    p.leaf_max, p.sah_bins, p.depth_cap = leaf_max, bins, depth_cap
    info = sc_scene_info()
    _check(lib.sc_bvh_build_host(tris.ctypes.data_as(C.c_void_p), n, C.byref(p), C.byref(hs),
                                 C.byref(info)), "sc_bvh_build_host")
    ni = info.n_inner
    return {"cbox": out["cbox"][:ni], "cref": out["cref"][:ni], "range": out["range"][:ni],
            "perm": out["perm"][:n], "n_inner": ni, "depth": info.depth, "root": info.root_ref}


@dataclass
class TraceResult:
    hits: "object"            # torch.int32 [n, 4]: prim, t bits, box tests, tri tests
    extra: "object" = None    # torch.int32 [n, 2]: mask tests, mask culls

    def numpy(self):
        h = self.hits.cpu().numpy()
        out = {"prim": h[:, 0].view(np.uint32).copy(), "t": h[:, 1].view(np.float32).copy(),
               "box_tests": h[:, 2].view(np.uint32).copy(), "tri_tests": h[:, 3].view(np.uint32).copy()}
        if self.extra is not None:
            e = self.extra.cpu().numpy()
            out["mask_tests"] = e[:, 0].view(np.uint32).copy()
            out["mask_culls"] = e[:, 1].view(np.uint32).copy()
        return out


class Scene:
    """A built scene (BVH + masks + codebook) on the context's device."""

    def __init__(self, ctx: Context, tris, *, R: int = 6, mode: str = "raw", K: int = 4096,
                 leaf_max: int = 4, bins: int = 32, depth_cap: int = 64, delta: float = 0.0,
                 origin_bound: float = 0.0, placement=None, width: int = 2, approx_levels: int = 0,
                 bit_table: bool = False, mask_slots: str = "all", quantise: bool = False, mask_test_max: int = 0,
                 stream=None):
        import torch
        lib = load()
        self.ctx = ctx
        if mask_slots not in ("all", "leaves"):
            raise ValueError("mask_slots must be 'all' or 'leaves'")
        if not isinstance(tris, torch.Tensor):
            tris = torch.from_numpy(np.ascontiguousarray(tris, np.float32))
        with _on_stream(stream):
            tris = tris.to(device=f"cuda:{ctx.device}", dtype=torch.float32).contiguous()
        n = tris.shape[0]
        p = sc_build_params()
        lib.sc_build_params_default(C.byref(p))
        p.R, p.leaf_max, p.sah_bins, p.depth_cap = R, leaf_max, bins, depth_cap
        p.mode, p.codebook_size = MODES[mode], K
        p.delta, p.origin_bound = delta, origin_bound
        p.width = width
        p.approx_levels = approx_levels
        p.bit_table = int(bit_table)
        p.mask_slots = 1 if mask_slots == "leaves" else 0
        p.quantise = 1 if quantise else 0
        p.mask_test_max = mask_test_max
        self._placement = None
        if placement is not None:
            self._placement = np.ascontiguousarray(placement, np.uint8)
            p.mask_placement = self._placement.ctypes.data_as(C.c_void_p)
            p.placement_len = self._placement.size
        h = C.c_void_p()
        _check(lib.sc_scene_build(ctx.handle, _ptr(tris) if n else None, n, C.byref(p),
                                  _stream_ptr(stream), C.byref(h)), "sc_scene_build")
        self.handle = h
        info = sc_scene_info()
        _check(lib.sc_scene_get_info(h, C.byref(info)), "sc_scene_get_info")
        self.info = {f: getattr(info, f) for f, _ in sc_scene_info._fields_}

    def close(self):
        if getattr(self, "handle", None):
            load().sc_scene_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def export(self) -> dict:
        """Host copies of the BVH, exact masks, codebook and indices."""
        I = self.info
        ni, n, W, K = I["n_inner"], I["n_tris"], I["words"], I["codebook_size"]
        out = {
            "cbox": np.zeros((max(ni, 1), 12), np.float32), "cref": np.zeros((max(ni, 1), 2), np.uint32),
            "range": np.zeros((max(ni, 1), 2), np.uint32), "perm": np.zeros(max(n, 1), np.uint32),
            "masks": np.zeros((max(2 * ni, 1), W), np.uint64),
            "codebook": np.zeros((max(K, 1), W), np.uint64), "cidx": np.zeros(max(2 * ni, 1), np.uint16),
        }
        hs = sc_scene_host(*(out[k].ctypes.data_as(C.c_void_p) for k in
                             ("cbox", "cref", "range", "perm", "masks", "codebook", "cidx")))
        _check(load().sc_scene_export(self.handle, C.byref(hs)), "sc_scene_export")
        out["cbox"], out["cref"], out["range"] = out["cbox"][:ni], out["cref"][:ni], out["range"][:ni]
        out["perm"], out["masks"], out["cidx"] = out["perm"][:n], out["masks"][:2 * ni], out["cidx"][:2 * ni]
        out["codebook"] = out["codebook"][:K]
        return out

    def export4(self) -> dict:
        """Host copies of a 4-wide scene's nodes: box4 [n4, 4, 6], ref4 and src4 [n4, 4]."""
        n4 = self.info["n_nodes"]
        out = {"box4": np.zeros((max(n4, 1), 4, 6), np.float32), "ref4": np.zeros((max(n4, 1), 4), np.uint32),
               "src4": np.zeros((max(n4, 1), 4), np.uint32)}
        _check(load().sc_scene_export4(self.handle, *(out[k].ctypes.data_as(C.c_void_p)
                                                       for k in ("box4", "ref4", "src4"))), "sc_scene_export4")
        return {k: v[:n4] for k, v in out.items()}

    def export_bit_table(self) -> np.ndarray:
        """Host copy of the 2-D bit table: uint32 [R^6, K/32]."""
        R, K = self.info["R"], self.info["codebook_size"]
        out = np.zeros((R ** 6, K // 32), np.uint32)
        _check(load().sc_scene_export_bit_table(self.handle, out.ctypes.data_as(C.c_void_p)),
               "sc_scene_export_bit_table")
        return out

    def features(self, stream=None):
        """Per-slot placement features, device float32 [2*n_inner, 12]."""
        import torch
        S = 2 * self.info["n_inner"]
        with _on_stream(stream):
            out = torch.empty((max(S, 1), 12), dtype=torch.float32, device=f"cuda:{self.ctx.device}")
            _check(load().sc_slot_features(self.handle, _ptr(out), _stream_ptr(stream)), "sc_slot_features")
        return out[:S]

    def trace(self, rays, *, cull: bool = True, shadow: bool = False, extra: bool = True, sort: bool = False,
              slot_fp=None, hits=None, extra_out=None, stream=None) -> TraceResult:
        """Trace device rays [n, 8] float32; results stay on the device."""
        import torch
        dev = f"cuda:{self.ctx.device}"
        if not isinstance(rays, torch.Tensor):
            rays = torch.from_numpy(np.ascontiguousarray(rays, np.float32))
        with _on_stream(stream):
            rays = rays.to(device=dev, dtype=torch.float32).contiguous()
            n = rays.shape[0]
            if hits is None:
                hits = torch.empty((max(n, 1), 4), dtype=torch.int32, device=dev)
            if extra and extra_out is None:
                extra_out = torch.empty((max(n, 1), 2), dtype=torch.int32, device=dev)
            flags = ((SC_TRACE_CULL if cull else 0) | (SC_TRACE_SHADOW if shadow else 0) |
                     (SC_TRACE_SORT if sort else 0))
            _check(load().sc_trace(self.handle, _ptr(rays), n, flags, _ptr(hits),
                                   _ptr(extra_out) if extra else None, _ptr(slot_fp),
                                   _stream_ptr(stream)), "sc_trace")
        return TraceResult(hits[:n], extra_out[:n] if extra else None)

    def ray_order(self, rays, stream=None):
        """Device int32 [n]: the order a sorted trace takes the rays in (sc_ray_order)."""
        import torch
        dev = f"cuda:{self.ctx.device}"
        if not isinstance(rays, torch.Tensor):
            rays = torch.from_numpy(np.ascontiguousarray(rays, np.float32))
        with _on_stream(stream):
            rays = rays.to(device=dev, dtype=torch.float32).contiguous()
            n = rays.shape[0]
            out = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
            _check(load().sc_ray_order(self.handle, _ptr(rays), n, _ptr(out), _stream_ptr(stream)),
                   "sc_ray_order")
        return out[:n]


def place_top(scores, n_place: int) -> np.ndarray:
    """uint8 placement marking the n_place highest scores (ties: lower index)."""
    scores = np.ascontiguousarray(scores, np.float32)
    out = np.zeros(max(scores.size, 1), np.uint8)
    _check(load().sc_place_top(scores.ctypes.data_as(C.c_void_p), scores.size, n_place,
                               out.ctypes.data_as(C.c_void_p)), "sc_place_top")
    return out[:scores.size]


class Batch:
    """Several scenes' rays traced by one persistent launch.

    ``items`` is a list of (scene, rays) pairs (rays: device float32 [n, 8]).
    ``graph=True`` records the launch once into a HIP graph; ``launch()``
    replays it. Output buffers are allocated here and stay bound to the batch.
    """

    def __init__(self, ctx: Context, items, *, cull: bool = True, shadow: bool = False,
                 extra: bool = True, graph: bool = True, slot_fp=None, sort: bool = False):
        import torch
        self.ctx = ctx
        dev = f"cuda:{ctx.device}"
        self.rays, self.hits, self.extra, self.slot_fp = [], [], [], []
        arr = (sc_batch_item * len(items))()
        for k, (scene, rays) in enumerate(items):
            if not isinstance(rays, torch.Tensor):
                rays = torch.from_numpy(np.ascontiguousarray(rays, np.float32))
            rays = rays.to(device=dev, dtype=torch.float32).contiguous()
            n = rays.shape[0]
            h = torch.empty((max(n, 1), 4), dtype=torch.int32, device=dev)
            e = torch.empty((max(n, 1), 2), dtype=torch.int32, device=dev) if extra else None
            fp = None if slot_fp is None else slot_fp[k]
            self.rays.append(rays)
            self.hits.append(h)
            self.extra.append(e)
            self.slot_fp.append(fp)
            arr[k] = sc_batch_item(scene.handle, rays.data_ptr() if n else None, n, h.data_ptr(),
                                   None if e is None else e.data_ptr(), None if fp is None else fp.data_ptr())
        self._arr = arr
        self._n = len(items)
        self.flags = ((SC_TRACE_CULL if cull else 0) | (SC_TRACE_SHADOW if shadow else 0) |
                      (SC_TRACE_SORT if sort else 0))
        self.handle = None
        if graph:
            h = C.c_void_p()
            _check(load().sc_batch_create(ctx.handle, arr, self._n, self.flags, C.byref(h)), "sc_batch_create")
            self.handle = h

    def launch(self, stream=None):
        if stream is not None:
            import torch
            cur = torch.cuda.current_stream(stream.device)
            if stream != cur:
                stream.wait_stream(cur)  # the rays were copied on the stream current at construction
        if self.handle is not None:
            _check(load().sc_batch_launch(self.handle, _stream_ptr(stream)), "sc_batch_launch")
        else:
            _check(load().sc_trace_batch(self.ctx.handle, self._arr, self._n, self.flags, _stream_ptr(stream)),
                   "sc_trace_batch")

    def results(self, k) -> TraceResult:
        n = self.rays[k].shape[0]
        return TraceResult(self.hits[k][:n], None if self.extra[k] is None else self.extra[k][:n])

    def close(self):
        if self.handle is not None:
            load().sc_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
