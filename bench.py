"""Benchmark: rays/s and (box + triangle) tests per ray, culled vs unculled, on one MI355X.

Default workload (the 12M-triangle curly-hair configuration): 12,000,000
float32 triangles (120k curly ribbon strands x 50 segments x 2 triangles,
width 5e-4, curl radius 3e-3, within 15 degrees of the (1,1,1) diagonal) and
8,000,000 incoherent bounce rays (cosine-diffuse rays leaving uniformly drawn
surface points). One step = one trace of the whole ray batch, rays and scene
resident in HBM. The headline value is the culled trace with 216-bit (R = 6)
masks compressed to a 4,096-entry conservative codebook (Sect. 3.2.2-3.2.3,
12-bit indices stored in 16 bits) on the 4-wide BVH (Sect. 3.2.4 node: four
child boxes and their codebook indices), each compressed-mask test answered by
one bit of the 2-D bit table of Sect. 3.2.2 (mode lut6w4b); the same masks
tested by fetching the codebook entry and the ray mask and ANDing them
(lut6w4, identical hits and counts), both on quantised child boxes, the plain
traversals (4-wide float and quantised boxes, binary) and 64-bit (R = 4) raw
masks are timed beside it. Each mode's
launch shape is the one the autotuner picked for it on this workload (stored
in MODES; --autotune re-runs the tuner, --sort switches Morton ray ordering);
results never depend on it. Other workloads: hair_1m (1M-triangle helical
strands, 4.1M primary + surface rays, raw masks), batch64, placement, approx.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--modes lut6w4,nonew4q,...]
                    [--no-cpu-baseline] [--cpu-seconds S] [--autotune | --tune b,s,c,p,w,o,q,g,f]
                    [--workload curly_12m|hair_1m|batch64|placement|approx] [--sort stored|0|1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "rays/sec and node+triangle tests/ray, culled vs unculled, 1 MI355X"
HBM_PEAK_GBS = 8000.0
RAY_BYTES, HIT_BYTES, EXTRA_BYTES, TRI_BYTES = 32, 16, 8, 48

# HBM-side bytes per trace launch from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE, each scaled by the
# same counter's reading for a 1 GiB plain copy (FETCH x2.0, WRITE x1.0). Valid only for the traversal
# kernel source whose SHA-256 starts with this prefix; otherwise traffic is reported as null.
MEASURED_TRAFFIC = {"source_sha256_16": "2995473634153956",
                    "curly_12m": {"lut6w4b": 69.73e9, "nonew4q": 43.01e9, "raw4w4q": 42.41e9, "lut6w4": 49.98e9},
                    "hair_1m": {"raw6w4": 16.85e9, "raw6w4q": 19.74e9, "raw4w4q": 13.02e9, "lut6w4b": 19.57e9,
                                "nonew4q": 11.48e9}}
TRACE_SOURCE = os.path.join(ROOT, "paper_2305_08343_amd", "csrc", "kernels_trace.hip")

# width 2: binary nodes (node_bytes per visit); width 4: 4-wide nodes of Sect. 3.2.4 (child records of
# 32 bytes, raw masks in their own array, mask_bytes per mask test). tune = (block, stack, chunk, parts,
# waves, sort) picked by the autotuner (bench.py --autotune) on this workload on one MI355X.
MODES = {
    "raw6w4": dict(mode="raw", R=6, cull=True, width=4, mask_bytes=32, tune=(256, 12, 1, 8, 6, 0, 0, 12, 12)),
    "raw4w4": dict(mode="raw", R=4, cull=True, width=4, mask_bytes=8, tune=(256, 12, 1, 8, 6, 0, 0, 12, 8)),
    "raw6w4l": dict(mode="raw", R=6, cull=True, width=4, mask_bytes=32, mask_slots="leaves", tune=(256, 12, 1, 8, 6, 0, 0, 12, 12)),
    "raw4w4l": dict(mode="raw", R=4, cull=True, width=4, mask_bytes=8, mask_slots="leaves", tune=(256, 12, 1, 8, 6, 0, 0, 12, 8)),
    "nonew4": dict(mode="none", R=6, cull=False, width=4, mask_bytes=0, tune=(128, 16, 1, 8, 6, 1, 0, 20, 20)),
    # quantised child boxes: 64-byte nodes, 16 bytes per child (6 plane bytes, ref, a quarter of corner + aux)
    "nonew4q": dict(mode="none", R=6, cull=False, width=4, mask_bytes=0, quantise=True, child_bytes=16,
                    tune=(256, 12, 1, 8, 6, 0, 0, 12, 12)),
    "raw6w4q": dict(mode="raw", R=6, cull=True, width=4, mask_bytes=32, quantise=True, child_bytes=16,
                    tune=(256, 12, 1, 8, 6, 0, 0, 12, 12)),
    "raw4w4q": dict(mode="raw", R=4, cull=True, width=4, mask_bytes=8, quantise=True, child_bytes=16,
                    tune=(256, 12, 1, 8, 6, 0, 0, 12, 8)),
    "raw4w4lq": dict(mode="raw", R=4, cull=True, width=4, mask_bytes=8, mask_slots="leaves", quantise=True,
                     child_bytes=16, tune=(256, 12, 1, 8, 6, 0, 0, 12, 8)),
    "lut6w4q": dict(mode="lut", R=6, cull=True, width=4, mask_bytes=0, K=4096, quantise=True, child_bytes=16,
                    tune=(256, 12, 1, 8, 0, 0, 1, 12, 12)),
    "lut4k256w4q": dict(mode="lut", R=4, cull=True, width=4, mask_bytes=0, K=256, quantise=True, child_bytes=16,
                        tune=(256, 8, 1, 8, 0, 0)),
    "lut6w4": dict(mode="lut", R=6, cull=True, width=4, mask_bytes=0, K=4096, tune=(256, 12, 1, 8, 6, 0)),
    "lut4k256w4": dict(mode="lut", R=4, cull=True, width=4, mask_bytes=0, K=256, tune=(256, 8, 1, 8, 0, 0)),
    "lut6k256w4": dict(mode="lut", R=6, cull=True, width=4, mask_bytes=0, K=256, tune=(256, 8, 1, 8, 6, 0)),
    "lut6w4b": dict(mode="lut", R=6, cull=True, width=4, mask_bytes=4, K=4096, bit_table=True, tune=(256, 12, 1, 8, 0, 0, 0, 8, 16)),
    "lut6w4bq": dict(mode="lut", R=6, cull=True, width=4, mask_bytes=4, K=4096, bit_table=True, quantise=True,
                     child_bytes=16, tune=(256, 12, 1, 8, 6, 0, 0, 12, 12)),
    "lut6k256w4b": dict(mode="lut", R=6, cull=True, width=4, mask_bytes=4, K=256, bit_table=True, tune=(256, 12, 1, 8, 6, 0)),
    "lut4k256w4b": dict(mode="lut", R=4, cull=True, width=4, mask_bytes=4, K=256, bit_table=True, tune=(256, 12, 1, 8, 0, 0)),
    "raw6": dict(mode="raw", R=6, cull=True, width=2, node_bytes=128, tune=(256, 12, 1, 8, 6, 1, 0, 12, 32)),
    "none": dict(mode="none", R=6, cull=False, width=2, node_bytes=64, tune=(256, 12, 1, 8, 0, 1, 0, 24, 20)),
    "raw4": dict(mode="raw", R=4, cull=True, width=2, node_bytes=128, tune=(256, 8, 1, 8, 0, 0)),
    "lut6": dict(mode="lut", R=6, cull=True, width=2, node_bytes=64, K=4096),
    "lut6k256": dict(mode="lut", R=6, cull=True, width=2, node_bytes=64, K=256),
    "lut4k256": dict(mode="lut", R=4, cull=True, width=2, node_bytes=64, K=256),
}
CHILD_BYTES_W4 = 32  # 24-byte box + 4-byte ref + 4 bytes of the node's aux word, per tested child

# Launch shapes the autotuner picked on the 12M-triangle curly workload (8M incoherent rays), where
# they differ from the hair_1m ones above.
CURLY_TUNE = {
    "lut6w4": (256, 12, 1, 8, 6, 1, 0, 12, 12),
    "lut6w4q": (256, 12, 1, 8, 0, 1, 1, 12, 12),
    "nonew4": (128, 16, 1, 8, 6, 1, 0, 20, 20),
    "nonew4q": (256, 12, 1, 8, 6, 1, 0, 12, 12),
    "none": (256, 12, 1, 8, 0, 1, 0, 24, 20),
    "raw4w4": (256, 12, 1, 8, 6, 1, 0, 12, 8),
    "raw4w4q": (256, 12, 1, 8, 6, 1, 0, 12, 8),
    "raw4w4l": (256, 12, 1, 8, 6, 1, 0, 12, 8),
    "raw6w4": (256, 12, 1, 8, 6, 1, 0, 12, 12),
    "lut6w4b": (256, 12, 1, 8, 6, 1, 0, 12, 24),
    "lut6w4bq": (256, 12, 1, 8, 6, 1, 0, 12, 12),
}


def mode_spec(name):
    """MODES[name]; "base@N" is mode base built with mask_test_max N: masks (raw, or the codebook
    entry a slot points to) with more than N set bits pass untested."""
    if "@" in name:
        base, limit = name.split("@")
        return dict(MODES[base], test_max=int(limit))
    return MODES[name]


def stored_tune(name, workload):
    """The launch shape bench.py uses for mode `name` on `workload` (a "base@N" mode: base's)."""
    if workload == "curly_12m" and name in CURLY_TUNE:
        return CURLY_TUNE[name]
    base = name.split("@")[0]
    if workload == "curly_12m" and base in CURLY_TUNE:
        return CURLY_TUNE[base]
    return MODES[base].get("tune", ())


def measured_traffic(mode, workload):
    import hashlib
    with open(TRACE_SOURCE, "rb") as f:
        h = hashlib.sha256(f.read()).hexdigest()[:16]
    if h != MEASURED_TRAFFIC["source_sha256_16"]:
        return None
    return MEASURED_TRAFFIC.get(workload, {}).get(mode)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(box_tests, tri_tests, mask_tests, n_rays, spec):
    """Bytes one trace launch must move: rays in, hits and mask counters out,
    one triangle record per triangle test, and the nodes: for binary nodes
    one node line per inner-node visit (two slab tests each); for 4-wide
    nodes one 32-byte child record per slab test plus one raw mask per mask
    test (or, with the 2-D bit table, the 4-byte word a test reads: the table
    is larger than an L2). The ray-mask LUT and the codebook are cache-resident
    by design and not counted."""
    tests = box_tests.sum(dtype=np.float64)
    if spec["width"] == 2:
        nodes = tests / 2.0 * spec["node_bytes"]
    else:
        nodes = tests * spec.get("child_bytes", CHILD_BYTES_W4) + mask_tests.sum(dtype=np.float64) * spec["mask_bytes"]
    return (n_rays * (RAY_BYTES + HIT_BYTES + EXTRA_BYTES) + nodes
            + tri_tests.sum(dtype=np.float64) * TRI_BYTES)


def hbm_probe(gib=2, reps=5):
    """Achievable HBM bandwidth: a plain device copy of `gib` GiB (read + write), best of `reps`."""
    import torch
    src = torch.ones(gib * 2 ** 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = None
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        best = ms if best is None else min(best, ms)
    bytes_moved = 2 * src.numel() * 4
    del src, dst
    return bytes_moved / (best * 1e-3) / 1e9


def time_mode(ctx, tris, rays_dev, name, spec, steps, warmup, autotune=False, workload="hair_1m"):
    import torch
    from paper_2305_08343_amd import binding, tune
    t0 = time.perf_counter()
    scene = binding.Scene(ctx, tris, R=spec["R"], mode=spec["mode"], K=spec.get("K", 4096), width=spec["width"],
                          bit_table=spec.get("bit_table", False), mask_slots=spec.get("mask_slots", "all"),
                          quantise=spec.get("quantise", False), mask_test_max=spec.get("test_max", 0))
    build_s = time.perf_counter() - t0
    n = rays_dev.shape[0]
    hits = torch.empty((n, 4), dtype=torch.int32, device=rays_dev.device)
    extra = torch.empty((n, 2), dtype=torch.int32, device=rays_dev.device)
    tuned = None
    if autotune:
        # shapes are compared on the whole ray set: on a subsample the persistent grid's drain weighs
        # more and the tuner's picks run slower on every ray
        key = f"{workload}|{name}|{tris.shape[0]}|{n}"
        lut = spec["mode"] == "lut" and not spec.get("bit_table", False)
        cfg, entry = tune.tuned(ctx, key, lambda: scene.trace(rays_dev, cull=spec["cull"], hits=hits,
                                                              extra_out=extra), log=log,
                                cands=tune.candidates(lut=lut))
        tuned = {"config": list(cfg), "seconds": entry.get("seconds")}
    res = scene.trace(rays_dev, cull=spec["cull"], hits=hits, extra_out=extra).numpy()
    for _ in range(warmup):
        scene.trace(rays_dev, cull=spec["cull"], hits=hits, extra_out=extra)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t_start = time.perf_counter()
    for k in range(steps):
        ev[k][0].record(stream)
        scene.trace(rays_dev, cull=spec["cull"], hits=hits, extra_out=extra)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    kernel_ms = np.array([a.elapsed_time(b) for a, b in ev])
    box, tri = res["box_tests"], res["tri_tests"]
    alg = algorithmic_bytes(box, tri, res["mask_tests"], n, spec)
    info = scene.info
    out = {
        "rays_per_s": n * steps / wall,
        "ms_per_step": 1e3 * wall / steps,
        "kernel_ms_mean": float(kernel_ms.mean()),
        "kernel_ms_min": float(kernel_ms.min()),
        "box_tests_per_ray": float(box.mean()),
        "tri_tests_per_ray": float(tri.mean()),
        "tests_per_ray": float((box.sum(dtype=np.float64) + tri.sum(dtype=np.float64)) / n),
        "mask_tests_per_ray": float(res["mask_tests"].mean()),
        "mask_culls_per_ray": float(res["mask_culls"].mean()),
        "hit_fraction": float((res["prim"] != 0xFFFFFFFF).mean()),
        "alg_bytes_per_launch": alg,
        "alg_gbs": alg / (kernel_ms.mean() * 1e-3) / 1e9,
        "build_s": build_s,
        "build_ms": {k: info[k] for k in ("ms_bvh", "ms_masks", "ms_codebook", "ms_compress")},
        "n_inner": info["n_inner"], "n_nodes": info["n_nodes"], "width": info["width"], "depth": info["depth"],
        "tune": ctx.get_tune(), "autotune": tuned,
        "scene_mbytes": info["device_bytes"] / 2 ** 20,
    }
    scene.close()
    return out, res


def cpu_model():
    """The host CPU's model name as lscpu reports it (else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        f = {k.strip(): v.strip() for k, v in (l.split(":", 1) for l in out.splitlines() if ":" in l)}
        if f.get("Model name"):
            # a virtual machine may report the bare family name; the family / model numbers identify the part
            ids = ", ".join(f"{k.lower()} {f[k]}" for k in ("CPU family", "Model", "Stepping") if f.get(k))
            return f"{f['Model name']} ({ids})" if ids else f["Model name"]
    except (OSError, subprocess.SubprocessError, ValueError):
        pass
    try:
        with open("/proc/cpuinfo") as f:
            return next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        return ""


def cpu_baseline(tris, rays, target_s, spec):
    """The oracle as it stands, on this host's cores, in the headline mode's configuration (mask
    resolution, raw or codebook-compressed masks, binary or 4-wide BVH, exact or quantised child
    boxes), traversal only, on an every-k-th ray sample sized to about target_s seconds."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    R, mode, width = spec["R"], spec["mode"], spec["width"]
    quant = spec.get("quantise", False)
    t0 = time.perf_counter()
    bvh = oracle.bvh_build(tris)
    ob, delta = oracle.default_bounds(tris)
    b4 = oracle.bvh4_collapse(bvh) if width == 4 else None
    if quant:
        b4 = oracle.decoded_bvh4(b4, oracle.quantise4(b4))
        bvh = oracle.with_slot_boxes(bvh, b4)
    kw = dict(mode=mode, R=R, origin_bound=ob, test_max=spec.get("test_max", 0))
    if mode != "none":
        if spec.get("approx_levels"):
            masks = oracle.approx_masks(tris, bvh, R, delta, spec["approx_levels"])
        else:
            masks = oracle.object_masks(tris, bvh, R, delta, nthreads=cores)
        if spec.get("mask_slots") == "leaves":
            masks = oracle.leaf_slot_masks(masks, bvh, R)
        if mode == "lut":
            cb, idx = oracle.compress(masks, bvh.slot_boxes(), R, spec.get("K", 4096))
            kw.update(codebook=cb, cidx=idx)
        else:
            kw.update(masks=masks)
        if mode == "sparse":
            kw.update(placed=spec["placed"])
        kw["lut"] = oracle.raymask_lut(R)
    setup = time.perf_counter() - t0

    def run(sample, nthreads):
        if b4 is not None:
            return oracle.trace4(tris, bvh, b4, sample, nthreads=nthreads, **kw)
        return oracle.trace(tris, bvh, sample, nthreads=nthreads, **kw)

    # one thread on rays spread evenly over the batch (rays/s per core)
    k1 = max(1, rays.shape[0] // 16384)
    first = rays[::k1][:16384]
    t0 = time.perf_counter()
    run(first, 1)
    one = first.shape[0] / (time.perf_counter() - t0)

    probe = rays[::4096]
    t0 = time.perf_counter()
    run(probe, cores)
    dt = max(time.perf_counter() - t0, 1e-4)
    want = int(min(rays.shape[0], max(probe.shape[0], probe.shape[0] * target_s / dt)))
    step = max(1, rays.shape[0] // want)
    sample = rays[::step]
    t0 = time.perf_counter()
    run(sample, cores)
    dt = time.perf_counter() - t0
    # untimed: how deep each sampled ray's stack gets (entries beneath the visited node, the stack
    # the GPU kernel keeps in LDS up to the launch shape's depth and in private memory beyond it)
    deep, refs = None, None
    if b4 is not None:
        h = oracle.trace4(tris, bvh, b4, sample, nthreads=cores, stack_depth=True, codebook_refs=(mode == "lut"),
                          **kw)
        deep, refs = h.deepest, h.cb_refs
    masks_txt = ("no masks (plain traversal)" if mode == "none" else
                 f"{'LUT K=' + str(spec.get('K', 4096)) if mode == 'lut' else mode} masks R={R}"
                 f"{' on %d placed slots' % int(np.count_nonzero(spec['placed'])) if mode == 'sparse' else ''}"
                 f"{' built by Alg. 2 at L = %d' % spec['approx_levels'] if spec.get('approx_levels') else ''}"
                 f"{' on leaf slots' if spec.get('mask_slots') == 'leaves' else ''}"
                 f"{', masks of more than %d set bits untested' % spec['test_max'] if spec.get('test_max') else ''}"
                 f", culled")
    what = f"{masks_txt}, {'4-wide' if width == 4 else 'binary'} BVH{' with quantised child boxes' if quant else ''}"
    out = {"value": sample.shape[0] / dt, "unit": "rays/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(), "rays_timed": int(sample.shape[0]), "seconds_timed": dt,
            "one_thread": {"value": one, "unit": "rays/s",
                           "sample": f"every {k1}th ray ({first.shape[0]:,} rays), 1 thread"},
            "sample": (f"all {rays.shape[0]:,} rays" if step == 1 else
                       f"every {step}th ray of the {rays.shape[0]:,} ({sample.shape[0]:,} rays)") +
                      f", {what}; {dt:.1f} s of traversal on {cores} threads; oracle BVH, mask and codebook "
                      f"set-up {setup:.1f} s not timed"}
    if refs is not None:
        out["codebook_refs"] = codebook_ref_report(refs, R)
    return out, deep


def codebook_ref_report(refs, R):
    """How the sample's mask tests spread over the codebook entries: the share of tests that read the
    most-read k entries (what an LDS copy of k entries, k * entry bytes, would serve)."""
    r = np.sort(np.asarray(refs, np.float64))[::-1]
    total = float(r.sum())
    cum = np.cumsum(r) / max(total, 1.0)
    words = (R ** 3 + 63) // 64
    return {"tests": int(total), "entries": int(r.size), "entries_read": int((r > 0).sum()),
            "entry_bytes": 8 * words,
            "share_of_tests_in_most_read": {str(k): float(cum[min(k, r.size) - 1]) for k in (16, 64, 256, 1024)
                                            if r.size}}


def stack_report(deep, lds_entries):
    """Stack depth of the sampled rays against the launch shape's LDS stack."""
    d = np.asarray(deep, np.int64)
    return {"lds_entries": int(lds_entries), "rays_sampled": int(d.size), "max_entries": int(d.max()),
            "mean_deepest": float(d.mean()), "p99_deepest": float(np.percentile(d, 99)),
            "frac_rays_beyond_lds": float((d > lds_entries).mean()),
            "source": "oracle 4-wide traversal of the cpu_baseline sample (the same visit sequence as the kernel)"}


def run_batch64(args, ctx):
    """64 scenes of uneven size in one persistent launch replayed from a HIP graph,
    against the same scenes traced one launch per scene."""
    import torch
    from paper_2305_08343_amd import binding, scenes, tune
    t0 = time.perf_counter()
    specs = scenes.batch_specs(64)
    data = [scenes.batch_scene(sp) for sp in specs]
    n_tris = sum(t.shape[0] for t, _ in data)
    n_rays = sum(r.shape[0] for _, r in data)
    log(f"batch64: {n_tris} tris, {n_rays} rays generated in {time.perf_counter() - t0:.1f}s")
    out = {}
    for mname in args.modes.split(","):
        spec = mode_spec(mname)
        t0 = time.perf_counter()
        built = [binding.Scene(ctx, t, R=spec["R"], mode=spec["mode"], K=spec.get("K", 4096), width=spec["width"],
                               quantise=spec.get("quantise", False), mask_slots=spec.get("mask_slots", "all"),
                               mask_test_max=spec.get("test_max", 0))
                 for t, _ in data]
        rays = [torch.from_numpy(r).cuda() for _, r in data]
        build_s = time.perf_counter() - t0
        direct = binding.Batch(ctx, list(zip(built, rays)), cull=spec["cull"], graph=False)
        key = f"batch64|{mname}|{n_tris}|{n_rays}"
        # batched launches take rays in descriptor order (no sorting); leaf and refill gathering
        # from the values that won on the single-scene workloads, to keep the search short
        cfg, entry = tune.tuned(ctx, key, direct.launch, log=log,
                                cands=[c for c in tune.candidates() if c[5] == 0 and c[7] in (12, 20)
                                       and c[8] in (12, 24)])
        graph = binding.Batch(ctx, list(zip(built, rays)), cull=spec["cull"], graph=True)
        hits = [torch.empty((max(r.shape[0], 1), 4), dtype=torch.int32, device="cuda") for r in rays]

        def per_scene():
            for s_, r_, h_ in zip(built, rays, hits):
                s_.trace(r_, cull=spec["cull"], hits=h_, extra=False)

        res = {}
        stream = torch.cuda.current_stream()
        for name, fn in (("graph_batch", graph.launch), ("per_scene_launches", per_scene)):
            for _ in range(args.warmup):
                fn()
            torch.cuda.synchronize()
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(args.steps)]
            t1 = time.perf_counter()
            for k in range(args.steps):
                ev[k][0].record(stream)
                fn()
                ev[k][1].record(stream)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t1) / args.steps
            res[name] = {"ms_per_step": dt * 1e3, "rays_per_s": n_rays / dt,
                         "launch_ms_mean": float(np.mean([a.elapsed_time(b) for a, b in ev]))}
        graph.launch()
        per_scene()
        torch.cuda.synchronize()
        same = all((graph.hits[k][:r.shape[0]].cpu().numpy() == hits[k][:r.shape[0]].cpu().numpy()).all()
                   for k, r in enumerate(rays) if r.shape[0])
        tests = sum(float(graph.hits[k][:r.shape[0], 2:4].sum().item()) for k, r in enumerate(rays))
        # algorithmic bytes of one batched launch: the single-scene byte model summed over the scenes,
        # from the batch's own per-ray counters
        alg = 0.0
        for k, r in enumerate(rays):
            n_k = r.shape[0]
            if not n_k:
                continue
            tr = graph.results(k).numpy()
            alg += algorithmic_bytes(tr["box_tests"], tr["tri_tests"], tr["mask_tests"], n_k, spec)
        res.update({"tune": list(cfg), "tune_seconds": entry.get("seconds"), "build_s": build_s,
                    "results_equal_per_scene": bool(same), "tests_per_ray": tests / n_rays,
                    "alg_bytes_per_launch": alg,
                    "alg_gbs": alg / (res["graph_batch"]["launch_ms_mean"] * 1e-3) / 1e9})
        log(f"batch64 {mname}: graph {res['graph_batch']['rays_per_s'] / 1e6:.1f} Mrays/s, per-scene "
            f"{res['per_scene_launches']['rays_per_s'] / 1e6:.1f} Mrays/s, tune {cfg}")
        out[mname] = res
        graph.close()
        direct.close()
        for s_ in built:
            s_.close()
    head_name = args.modes.split(",")[0]
    head = out[head_name]
    line = {
        "metric": METRIC, "value": head["graph_batch"]["rays_per_s"], "unit": "rays/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["graph_batch"]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch64: 64 scenes (10k-500k tris, strands/thin quads/isotropic), 16k-2M rays "
                               f"each (half pinhole, half random), one persistent launch replayed from a HIP graph, "
                               f"mode {head_name}",
                   "n_tris": n_tris, "n_rays": n_rays},
        "tests_per_ray": head["tests_per_ray"],
        "roofline": {"bound": "hbm", "achieved": head["alg_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": head["alg_gbs"] / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "trace_kernel (batched, one graph launch)",
                     "kernel_ms": head["graph_batch"]["launch_ms_mean"],
                     "alg_bytes_per_launch": head["alg_bytes_per_launch"],
                     "alg_bytes_per_ray": head["alg_bytes_per_launch"] / n_rays},
        "modes": out,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, every scene)")
        line["cpu_baseline"] = batch_cpu_baseline(data, mode_spec(head_name))
    print(json.dumps(line), flush=True)


def batch_cpu_baseline(data, spec):
    """The oracle on every ray of the batch's scenes, one scene after another (a few seconds of
    traversal in all): rays/s over the whole batch."""
    rays_t, secs, setup, parts, o = 0, 0.0, 0.0, [], None
    for k, (tris, rays) in enumerate(data):
        t0 = time.perf_counter()
        o, _ = cpu_baseline(tris, rays, 1e9, spec)  # no time limit: every ray
        rays_t += o["rays_timed"]
        secs += o["seconds_timed"]
        setup += time.perf_counter() - t0 - o["seconds_timed"]
        if o["rays_timed"] < rays.shape[0]:
            parts.append(f"scene {k}: {o['rays_timed']:,} of {rays.shape[0]:,} rays")
    total = sum(r.shape[0] for _, r in data)
    return {"value": rays_t / secs, "unit": "rays/s", "cores": o["cores"], "kind": "oracle",
            "cpu_model": o["cpu_model"], "rays_timed": rays_t, "seconds_timed": secs,
            "sample": f"the {len(data)} scenes one after another, {rays_t:,} of the {total:,} rays "
                      f"({'all' if not parts else 'every-k-th samples in ' + '; '.join(parts)}), "
                      f"{o['sample'].split(', ', 1)[1].split(';')[0]}; {secs:.1f} s of traversal on {o['cores']} "
                      f"threads; oracle set-up and single-thread probes {setup:.1f} s not timed"}


def run_placement(args, ctx):
    """Learned mask placement: the MLP is trained on the GPU on per-slot
    false-positive counts of generated strand / curly / thin-quad scenes
    (100k-2M tris), then places R = 6 masks at 0.5, 1 and 2 bytes per inner
    node on held-out 5M-tri scenes with 4M rays; compared with all masks, no
    masks, the SA x emptiness heuristic, random and true-count placement."""
    from paper_2305_08343_amd import placement, scenes
    t0 = time.perf_counter()
    specs = scenes.placement_specs(args.place_scenes)
    held = [scenes.placement_heldout(k) for k in range(args.place_heldout)]
    log(f"placement: {len(specs)} training scenes, {len(held)} held-out scenes")
    kept = []
    params, hist, res = placement.run_experiment(ctx, specs, held, log=log, placements_out=kept)
    total_s = time.perf_counter() - t0
    table = [[{k: v for k, v in e.__dict__.items()} for e in r] for r in res]
    head = {(e.name, e.beta): e for e in res[0]}[("learned", 1.0)]
    # the value's trace: sparse R = 6 masks (64-byte binary nodes, 32-byte side masks) on the held-out
    # hair scene; the timed traces write hits only
    n_rays = held[0][1].shape[0]
    alg = n_rays * (RAY_BYTES + HIT_BYTES) + n_rays * (head.box_per_ray / 2.0 * 64 + head.mask_per_ray * 32 +
                                                       head.tri_per_ray * TRI_BYTES)
    alg_gbs = alg / (head.ms * 1e-3) / 1e9
    line = {
        "metric": METRIC, "value": head.rays_per_s, "unit": "rays/s", "n_gpus": 1,
        "steps": 5, "warmup": 1, "ms_per_step": head.ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"placement: MLP 12-64-64-1 trained on {len(specs)} generated scenes "
                               "(100k-2M tris, 262,144 rays each), R=6 masks placed by predicted "
                               "false positives at 1 byte per inner node on a held-out 5M-tri hair "
                               "scene with 4M rays (value); all budgets and baselines in 'placement'",
                   "n_train_scenes": len(specs)},
        "tests_per_ray": head.tests_per_ray,
        "roofline": {"bound": "hbm", "achieved": alg_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": alg_gbs / HBM_PEAK_GBS, "traffic": None, "kernel": "trace_kernel (binary, sparse masks)",
                     "kernel_ms": head.ms, "alg_bytes_per_launch": alg, "alg_bytes_per_ray": alg / n_rays},
        "train_loss": hist, "seconds_total": total_s,
        "placement": table,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, learned placement at 1 byte per inner node)")
        spec = {"R": 6, "mode": "sparse", "width": 2, "placed": kept[0][("learned", 1.0)]}
        line["cpu_baseline"], _ = cpu_baseline(held[0][0], held[0][1], args.cpu_seconds, spec)
    print(json.dumps(line), flush=True)


def run_approx(args, ctx):
    """Approximate object masks (Sect. 3.2.1, Alg. 2) on the 1M-triangle hair workload: mask build time and
    culling (tests/ray, rays/s) for L = 1..5 and exact masks, R = 4 and 6, on the 4-wide BVH."""
    import torch
    from paper_2305_08343_amd import binding, scenes
    tris = scenes.scene_hair_1m(1)
    rays = scenes.rays_hair_1m(tris, 1)
    rays_dev = torch.from_numpy(rays).cuda()
    n = rays.shape[0]
    hits = torch.empty((n, 4), dtype=torch.int32, device="cuda")
    table = {}
    for R in (4, 6):
        for L in (1, 2, 3, 4, 5, 0):
            ctx.set_tune(*MODES[f"raw{R}w4"]["tune"])
            sc = binding.Scene(ctx, tris, R=R, mode="raw", width=4, approx_levels=L)
            ms_masks = sc.info["ms_masks"]
            ex = sc.trace(rays_dev, hits=hits, extra=True).extra.cpu().numpy()
            torch.cuda.synchronize()
            h = hits.cpu().numpy()
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(args.steps)]
            for a, b in evs:
                a.record()
                sc.trace(rays_dev, hits=hits, extra=False)
                b.record()
            torch.cuda.synchronize()
            ms = float(np.median([a.elapsed_time(b) for a, b in evs]))
            sc.close()
            tests = (h[:, 2].astype(np.float64).sum() + h[:, 3].astype(np.float64).sum()) / n
            key = f"R{R}_L{L if L else 'exact'}"
            # the timed traces write hits only: the byte model without the mask counters
            alg = algorithmic_bytes(h[:, 2].view(np.uint32), h[:, 3].view(np.uint32), ex[:, 0].view(np.uint32), n,
                                    mode_spec(f"raw{R}w4")) - n * EXTRA_BYTES
            table[key] = {"mask_build_ms": ms_masks, "tests_per_ray": tests, "trace_ms": ms,
                          "rays_per_s": n / (ms * 1e-3), "alg_bytes_per_launch": alg,
                          "alg_gbs": alg / (ms * 1e-3) / 1e9}
            log(f"approx {key}: masks {ms_masks:.2f} ms, {tests:.2f} tests/ray, {n / ms / 1e3:.1f} Mrays/s")
    for R in (4, 6):
        base = table[f"R{R}_L1"]
        for k, v in table.items():
            if k.startswith(f"R{R}_"):
                v["tests_ratio_vs_L1"] = v["tests_per_ray"] / base["tests_per_ray"]
                v["build_time_ratio_vs_L1"] = v["mask_build_ms"] / base["mask_build_ms"]
    head = table["R6_L3"]
    line = {
        "metric": METRIC, "value": head["rays_per_s"], "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": head["trace_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "approx: hair_1m (1,000,002 tris, 4,147,200 rays), 4-wide BVH, raw masks built by "
                               "Alg. 2 at L = 1..5 or exactly; value = R=6, L=3", "n_tris": int(tris.shape[0]),
                   "n_rays": n},
        "roofline": {"bound": "hbm", "achieved": head["alg_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": head["alg_gbs"] / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "trace_kernel (4-wide, raw R=6 masks)", "kernel_ms": head["trace_ms"],
                     "alg_bytes_per_launch": head["alg_bytes_per_launch"],
                     "alg_bytes_per_ray": head["alg_bytes_per_launch"] / n},
        "approx": table,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, R=6 masks by Alg. 2 at L=3)")
        spec = dict(mode_spec("raw6w4"))
        spec["approx_levels"] = 3
        line["cpu_baseline"], _ = cpu_baseline(tris, rays, args.cpu_seconds, spec)
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--modes", default="",
                    help="comma-separated MODES keys; the first is the headline (default per workload)")
    ap.add_argument("--autotune", action="store_true",
                    help="pick each mode's launch shape live with the autotuner instead of the stored one")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--tune", default="", help="block,stack,chunk,parts[,waves[,sort[,codebook[,gather[,refill]]]]] of the traversal launch")
    ap.add_argument("--workload", default="curly_12m",
                    choices=["curly_12m", "hair_1m", "batch64", "placement", "approx"])
    ap.add_argument("--sort", choices=["stored", "0", "1"], default="stored",
                    help="Morton ray ordering: as stored in each mode's launch shape, off, or on")
    ap.add_argument("--place-scenes", type=int, default=200)
    ap.add_argument("--place-heldout", type=int, default=2)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the library measures one GPU's "
                                   "share (rays shard across GPUs with no exchange)",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_2305_08343_amd import binding, scenes
    assert torch.cuda.is_available(), "bench needs a GPU"
    binding.load()

    if args.workload == "batch64":
        ctx = binding.Context(0)
        if not args.modes:
            args.modes = "raw4w4q,nonew4q,raw6,none"
        run_batch64(args, ctx)
        ctx.close()
        return
    if args.workload == "approx":
        ctx = binding.Context(0)
        run_approx(args, ctx)
        ctx.close()
        return
    if args.workload == "placement":
        ctx = binding.Context(0)
        run_placement(args, ctx)
        ctx.close()
        return
    t0 = time.perf_counter()
    if args.workload == "curly_12m":
        tris = scenes.scene_curly_12m(2)
        rays = scenes.rays_curly_12m(tris)
        if not args.modes:
            args.modes = "lut6w4b,lut6w4,lut6w4bq,lut6w4q,nonew4,nonew4q,none,raw4w4,raw4w4q,raw4w4l"
        desc = ("curly_12m: 12,000,000 tris (120k curly strands x 50 segments x 2 tris, width 5e-4, curl "
                "radius 3e-3, within 15 deg of the (1,1,1) diagonal), 8,000,000 incoherent bounce rays "
                "(cosine-diffuse rays from uniformly drawn surface points), SAH BVH (4-wide in the w4 modes), "
                "216-bit (R=6) masks LUT-compressed to a 4,096-entry conservative codebook in the lut6 modes, "
                "tested through the 2-D bit table in the b modes")
    else:
        tris = scenes.scene_hair_1m(1)
        rays = scenes.rays_hair_1m(tris, 1)
        if not args.modes:
            args.modes = "raw6w4,raw6w4q,raw6w4l,nonew4,nonew4q,none,raw6,raw4w4"
        desc = ("hair_1m: 1,000,002 tris (20k helical strands x 25 segments x 2 tris, "
                "width 1e-3, + ground plane), 4,147,200 rays (1920x1080 pinhole primaries + 2,073,600 "
                "uniform surface bounce rays: cosine-diffuse rays from uniformly drawn surface points, "
                "not from the primary hits), SAH BVH (binary; 4-wide in the w4 modes)")
    log(f"generated {tris.shape[0]} tris, {rays.shape[0]} rays in {time.perf_counter() - t0:.1f}s")
    ctx = binding.Context(0)
    autotune = args.autotune and not args.tune
    rays_dev = torch.from_numpy(rays).cuda()
    modes = [m for m in args.modes.split(",") if m]
    results, raw = {}, {}
    for m in modes:
        if args.tune:
            ctx.set_tune(*(int(x) for x in args.tune.split(",")))
        else:
            ctx.set_tune(*stored_tune(m, args.workload))
        if args.sort != "stored":
            t = ctx.get_tune()
            ctx.set_tune(t["block"], t["stack"], t["chunk"], t["parts"], t["waves"], int(args.sort), t["codebook"],
                         t["gather"], t["refill"])
        log(f"mode {m}: build{' + autotune' if autotune else ''} + {args.warmup} warmup + {args.steps} timed traces")
        results[m], raw[m] = time_mode(ctx, tris, rays_dev, m, mode_spec(m), args.steps, args.warmup, autotune,
                                       args.workload)
        log(f"mode {m}: {results[m]['rays_per_s'] / 1e6:.1f} Mrays/s, "
            f"{results[m]['tests_per_ray']:.2f} tests/ray, kernel {results[m]['kernel_ms_mean']:.3f} ms")
    head = modes[0]
    for m in modes:
        # unculled reference: the plain traversal of the same node width, and the plain binary BVH
        plain = ("nonew4q" if mode_spec(m).get("quantise") else "nonew4") if mode_spec(m)["width"] == 4 else "none"
        for key, ref in (("unculled", plain), ("plain_binary", "none")):
            if ref not in raw or ref == m:
                continue
            same = bool((raw[m]["prim"] == raw[ref]["prim"]).all() and
                        (raw[m]["t"].view(np.uint32) == raw[ref]["t"].view(np.uint32)).all())
            results[m][f"hits_equal_{key}"] = same
            results[m][f"tests_ratio_vs_{key}"] = results[m]["tests_per_ray"] / results[ref]["tests_per_ray"]
            results[m][f"speedup_vs_{key}"] = results[m]["rays_per_s"] / results[ref]["rays_per_s"]
    r = results[head]
    n_rays = int(rays.shape[0])
    traffic = measured_traffic(head, args.workload)
    probe_gbs = hbm_probe()
    log(f"HBM copy probe: {probe_gbs:.0f} GB/s")
    line = {
        "metric": METRIC, "value": r["rays_per_s"], "unit": "rays/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{desc}, mode {head}", "n_tris": int(tris.shape[0]),
                   "n_rays": int(rays.shape[0])},
        "tests_per_ray": r["tests_per_ray"],
        "roofline": {"bound": "hbm", "achieved": r["alg_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": r["alg_gbs"] / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "trace_kernel", "kernel_ms": r["kernel_ms_mean"], "launch_shape": r["tune"],
                     "alg_bytes_per_launch": r["alg_bytes_per_launch"],
                     "alg_bytes_per_ray": r["alg_bytes_per_launch"] / n_rays,
                     "roofline_rays_per_s": HBM_PEAK_GBS * 1e9 / (r["alg_bytes_per_launch"] / n_rays),
                     "traffic_gbs": (traffic / (r["kernel_ms_mean"] * 1e-3) / 1e9) if traffic else None,
                     "traffic_bytes_per_ray": (traffic / n_rays) if traffic else None,
                     "hbm_probe_gbs": probe_gbs},
        "modes": results,
        "tune": r["tune"],
    }
    if args.copy_probe_mib:
        src = torch.ones(args.copy_probe_mib * 2 ** 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        line["copy_probe_bytes"] = src.numel() * 4
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        line["cpu_baseline"], deep = cpu_baseline(tris, rays, args.cpu_seconds, mode_spec(head))
        if deep is not None:
            line["lds_stack"] = stack_report(deep, r["tune"]["stack"])
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
