"""The C-ABI library loads and exports every symbol include/subcull.h declares;
argument checks that happen before any HIP call (CPU-only)."""
import ctypes as C
import os
import re

import pytest

from paper_2305_08343_amd import binding as B

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                      "subcull.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sc_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_api():
    names = _declared()
    for must in ("sc_create", "sc_destroy", "sc_scene_build", "sc_scene_destroy", "sc_scene_get_info",
                 "sc_scene_export", "sc_trace", "sc_raymask_lut", "sc_compress_masks",
                 "sc_status_string", "sc_last_error", "sc_build_params_default", "sc_set_tune",
                 "sc_get_tune", "sc_trace_batch", "sc_batch_create", "sc_batch_launch",
                 "sc_batch_destroy", "sc_bvh_build_host", "sc_slot_features", "sc_mlp_forward",
                 "sc_mlp_backward", "sc_mlp_adam", "sc_place_top", "sc_ray_order",
                 "sc_scene_export4", "sc_scene_export_bit_table", "sc_trace_noalloc",
                 "sc_set_device_checks", "sc_get_check_flags", "sc_set_check_limits"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = B.load()
    for name in _declared():
        assert hasattr(lib, name), name
        assert name in B._SIGS, f"binding lacks a signature for {name}"


def test_params_default_and_status_strings():
    lib = B.load()
    p = B.sc_build_params()
    lib.sc_build_params_default(C.byref(p))
    assert (p.R, p.leaf_max, p.sah_bins, p.depth_cap, p.mode, p.codebook_size) == (6, 4, 32, 64, 1, 4096)
    assert p.delta == 0.0 and p.origin_bound == 0.0 and not p.mask_placement and p.width == 2
    for s, txt in [(0, b"ok"), (1, b"invalid argument"), (4, b"BVH depth cap exceeded")]:
        assert lib.sc_status_string(s) == txt


def test_struct_sizes_match_header_layout():
    # 15 uint32, 2 float, (4 bytes of padding) uint64, 4 double
    assert C.sizeof(B.sc_scene_info) == 60 + 8 + 4 + 8 + 32
    assert C.sizeof(B.sc_build_params) == 72
    assert C.sizeof(B.sc_scene_host) == 7 * 8
    assert C.sizeof(B.sc_tune) == 9 * 4


def test_null_arguments_rejected_before_hip():
    lib = B.load()
    assert lib.sc_create(0, None, None) == 1
    assert lib.sc_scene_build(None, None, 0, None, None, None) == 1
    assert b"non-NULL" in lib.sc_last_error()
    assert lib.sc_trace(None, None, 0, 0, None, None, None, None) == 1
    assert lib.sc_trace_noalloc(None, None, 0, 0, None, None, None, None) == 1
    assert lib.sc_scene_get_info(None, None) == 1
    assert lib.sc_scene_export(None, None) == 1
    assert lib.sc_raymask_lut(None, 6, None, None) == 1
    assert lib.sc_compress_masks(None, 6, None, 64, None, 0, None, None) == 1
    assert lib.sc_set_tune(None, None) == 1 and lib.sc_get_tune(None, None) == 1
    assert lib.sc_ray_order(None, None, 0, None, None) == 1
    assert lib.sc_scene_export4(None, None, None, None) == 1
    assert lib.sc_scene_export_bit_table(None, None) == 1
    assert lib.sc_trace_batch(None, None, 0, 0, None) == 1
    assert lib.sc_batch_create(None, None, 0, 0, None) == 1
    assert lib.sc_batch_launch(None, None) == 1 and lib.sc_batch_destroy(None) == 0
    assert lib.sc_set_device_checks(None, 1) == 1
    assert lib.sc_get_check_flags(None, None, 0) == 1
    assert lib.sc_set_check_limits(None, 0, 0, 0) == 1
    assert lib.sc_destroy(None) == 0 and lib.sc_scene_destroy(None) == 0


def test_mlp_constants_match_header():
    text = open(HEADER).read()
    assert int(re.search(r"#define SC_MLP_PARAMS (\d+)", text).group(1)) == B.SC_MLP_PARAMS
    assert int(re.search(r"#define SC_MLP_GRAD_PARTS (\d+)", text).group(1)) == B.SC_MLP_GRAD_PARTS
    assert "#define SC_MLP_WORK_FLOATS(n) ((size_t)(n) * 130 + (size_t)SC_MLP_GRAD_PARTS * SC_MLP_PARAMS)" in text
    assert B.mlp_work_floats(1000) == 1000 * 130 + B.SC_MLP_GRAD_PARTS * B.SC_MLP_PARAMS


def test_check_bits_match_header():
    text = open(HEADER).read()
    bits = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define (SC_CHECK_[A-Z]+) (\d+)u", text)}
    assert bits == {"SC_CHECK_NODE": B.SC_CHECK_NODE, "SC_CHECK_TRI": B.SC_CHECK_TRI,
                    "SC_CHECK_STACK": B.SC_CHECK_STACK, "SC_CHECK_INDEX": B.SC_CHECK_INDEX}
    assert len(set(bits.values())) == 4 and all(v & (v - 1) == 0 for v in bits.values())


def test_bad_build_params_rejected_before_hip():
    lib = B.load()
    p = B.sc_build_params()
    lib.sc_build_params_default(C.byref(p))
    fake_ctx = C.c_void_p(1)  # never dereferenced: parameter checks come first
    out = C.c_void_p()
    for field, value in [("R", 5), ("leaf_max", 0), ("leaf_max", 5), ("sah_bins", 1), ("depth_cap", 65),
                         ("mode", 9), ("width", 3), ("width", 0), ("approx_levels", 65), ("bit_table", 1)]:
        q = B.sc_build_params.from_buffer_copy(p)
        setattr(q, field, value)
        assert lib.sc_scene_build(fake_ctx, None, 0, C.byref(q), None, C.byref(out)) == 1, field
    q = B.sc_build_params.from_buffer_copy(p)
    q.mode, q.codebook_size = 2, 100
    assert lib.sc_scene_build(fake_ctx, None, 0, C.byref(q), None, C.byref(out)) == 1
    q = B.sc_build_params.from_buffer_copy(p)
    q.mode = 3
    assert lib.sc_scene_build(fake_ctx, None, 0, C.byref(q), None, C.byref(out)) == 1
    assert b"mask_placement" in lib.sc_last_error()
    q.width = 4
    q.mask_placement = C.c_void_p(1)
    assert lib.sc_scene_build(fake_ctx, None, 0, C.byref(q), None, C.byref(out)) == 1
    assert b"width 2" in lib.sc_last_error()
    assert lib.sc_scene_build(fake_ctx, None, 1 << 29, C.byref(p), None, C.byref(out)) == 1


def test_no_device_is_reported(monkeypatch):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    assert B.load().sc_create(0, None, C.byref(h)) == 2


def test_place_top_host():
    import numpy as np
    scores = np.array([0.5, 2.0, -1.0, 2.0, 0.5, 3.0], np.float32)
    assert list(B.place_top(scores, 3)) == [0, 1, 0, 1, 0, 1]
    assert list(B.place_top(scores, 4)) == [1, 1, 0, 1, 0, 1]  # tie at 0.5: lower slot first
    assert B.place_top(scores, 0).sum() == 0 and B.place_top(scores, 6).sum() == 6
    with pytest.raises(B.SubcullError):
        B.place_top(scores, 7)


def test_place_top_orders_nan_and_minus_infinity_last():
    import numpy as np
    scores = np.array([np.nan, 1.0, -np.inf, 0.0, np.nan], np.float32)
    assert list(B.place_top(scores, 2)) == [0, 1, 0, 1, 0]
    # NaN and -inf tie at the bottom: lower slot first
    assert list(B.place_top(scores, 3)) == [1, 1, 0, 1, 0]
    assert list(B.place_top(scores, 4)) == [1, 1, 1, 1, 0]


def test_placeable_moves_full_mask_slots_last():
    import numpy as np
    import torch
    from paper_2305_08343_amd import placement
    X = torch.zeros((4, 12))
    X[:, 6] = torch.tensor([0.5, 1.0, 0.1, 1.0])
    s = placement.placeable(np.array([1.0, 9.0, 2.0, 8.0], np.float32), X)
    assert list(B.place_top(s, 2)) == [1, 0, 1, 0]
