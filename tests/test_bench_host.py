"""Host-side checks of the benchmark's own logic (no GPU): the algorithmic byte model, the guard on
the measured-traffic table, the mode table and the stored launch shapes, and the report helpers."""
import hashlib
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _configs_from_header():
    # the (block, stack) pairs the library compiles, read from its internal header
    import re
    txt = open(os.path.join(ROOT, "paper_2305_08343_amd", "csrc", "internal.h")).read()
    body = re.search(r"kTraceConfigs\[\]\[2\] = \{(.*?)\};", txt).group(1)
    return {tuple(int(v) for v in m) for m in re.findall(r"\{(\d+),\s*(\d+)\}", body)}


def test_byte_model_binary_and_4_wide():
    box = np.array([10, 6], np.uint32)
    tri = np.array([3, 1], np.uint32)
    mask = np.array([4, 2], np.uint32)
    n = 2
    per_ray = bench.RAY_BYTES + bench.HIT_BYTES + bench.EXTRA_BYTES
    # binary: one node line per visit, two slab tests a visit
    spec2 = dict(width=2, node_bytes=64)
    assert bench.algorithmic_bytes(box, tri, mask, n, spec2) == n * per_ray + 16 / 2 * 64 + 4 * bench.TRI_BYTES
    # 4-wide: a child record per slab test plus the mask bytes of each mask test
    spec4 = dict(width=4, mask_bytes=8)
    assert bench.algorithmic_bytes(box, tri, mask, n, spec4) == \
        n * per_ray + 16 * bench.CHILD_BYTES_W4 + 6 * 8 + 4 * bench.TRI_BYTES
    spec4q = dict(width=4, mask_bytes=4, child_bytes=16)
    assert bench.algorithmic_bytes(box, tri, mask, n, spec4q) == n * per_ray + 16 * 16 + 6 * 4 + 4 * bench.TRI_BYTES


def test_measured_traffic_only_for_the_profiled_source():
    with open(bench.TRACE_SOURCE, "rb") as f:
        h = hashlib.sha256(f.read()).hexdigest()[:16]
    got = bench.measured_traffic("lut6w4b", "curly_12m")
    if h == bench.MEASURED_TRAFFIC["source_sha256_16"]:
        assert got == bench.MEASURED_TRAFFIC["curly_12m"]["lut6w4b"]
    else:
        assert got is None
    assert bench.measured_traffic("no-such-mode", "curly_12m") is None


def test_mode_table_is_consistent():
    configs = _configs_from_header()
    for name, m in bench.MODES.items():
        assert m["mode"] in ("none", "raw", "lut", "sparse"), name
        assert m["R"] in (4, 6), name
        assert m["width"] in (2, 4), name
        if m["width"] == 2:
            assert "node_bytes" in m, name
        else:
            assert "mask_bytes" in m, name
            if m.get("quantise"):
                assert m.get("child_bytes") == 16, name
        if m["mode"] == "lut":
            assert m["K"] % 64 == 0 and 64 <= m["K"] <= 4096, name
        if m.get("bit_table"):
            assert m["mode"] == "lut" and m["mask_bytes"] == 4, name
        if m["mode"] == "raw" and m["width"] == 4:
            assert m["mask_bytes"] == 8 * ((m["R"] ** 3 + 63) // 64), name
        t = m.get("tune", ())
        if t:
            assert (t[0], t[1]) in configs, (name, t)


def test_stored_launch_shapes_are_compiled_and_in_range():
    configs = _configs_from_header()
    for name, t in bench.CURLY_TUNE.items():
        assert name in bench.MODES, name
        block, stack, chunk, parts, waves, sort, codebook, gather, refill = t
        assert (block, stack) in configs, (name, t)
        assert 1 <= chunk <= 64 and 1 <= parts <= 8 and 0 <= waves <= 8
        assert sort in (0, 1) and codebook in (0, 1) and 0 <= gather <= 64 and 0 <= refill <= 64
        assert bench.stored_tune(name, "curly_12m") == t
    # elsewhere a mode's own shape; "base@N" modes take their base's
    assert bench.stored_tune("raw6w4", "hair_1m") == bench.MODES["raw6w4"]["tune"]
    assert bench.stored_tune("lut6w4b@40", "curly_12m") == bench.CURLY_TUNE["lut6w4b"]
    assert bench.mode_spec("lut6w4b@40")["test_max"] == 40


def test_report_helpers():
    r = bench.codebook_ref_report(np.array([0, 5, 3, 2] + [0] * 60, np.int64), 6)
    assert r["tests"] == 10 and r["entries"] == 64 and r["entries_read"] == 3 and r["entry_bytes"] == 32
    assert r["share_of_tests_in_most_read"]["16"] == 1.0
    s = bench.stack_report(np.array([3, 12, 13, 40]), 12)
    assert s["max_entries"] == 40 and s["frac_rays_beyond_lds"] == 0.5 and s["rays_sampled"] == 4


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    line = json.loads([x for x in r.stdout.splitlines() if x.startswith("{")][0])
    assert line["n_gpus"] == 2
