"""Pins of the oracle's mask compression (Sect. 3.2.2, 3.2.3, Eq. 2, Alg. 3).

* Alg. 3 (requirement LUTs + lowest set bit) returns the same index as the
  brute-force tightest-superset scan the paper compares against;
* every chosen entry is a conservative superset of the original mask;
* the codebook is sorted by set-bit count, holds the full mask, and its
  other entries are the most important patterns by SA(N) * O_m(N) / R^3;
* table counts and sizes follow from R and b = 8 (ceil(R^3 / b) tables of
  2^b rows).
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2305_08343_amd import scenes
from tests.conftest import popcount64

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_layout_facts.json")


def _full(R):
    m = np.zeros(oracle.words_for(R), np.uint64)
    for b in range(R ** 3):
        m[b >> 6] |= np.uint64(1) << np.uint64(b & 63)
    return m


def _is_superset(big, small):
    return ((small & ~big) == 0).all(axis=-1)


def _random_masks(rng, n, R, density):
    bits = rng.random((n, R ** 3)) < density
    W = oracle.words_for(R)
    out = np.zeros((n, W), np.uint64)
    for b in range(R ** 3):
        out[:, b >> 6] |= bits[:, b].astype(np.uint64) << np.uint64(b & 63)
    return out


@pytest.mark.parametrize("R,K", [(4, 256), (6, 256), (6, 4096)])
def test_alg3_equals_naive_on_scene(small_oracle, R, K):
    masks = small_oracle[f"masks{R}"]
    bvh = small_oracle["bvh"]
    cb = oracle.codebook(masks, bvh.slot_boxes(), R, K)
    req = oracle.req_luts(cb, R)
    assert req.shape == (-(-R ** 3 // 8), 256, K // 64)
    idx = oracle.alg3(masks, req, K, R)
    assert (idx == oracle.naive_search(masks, cb, R)).all()
    assert _is_superset(cb[idx], masks).all()


@pytest.mark.parametrize("seed", range(6))
def test_alg3_equals_naive_random_codebooks(seed):
    rng = np.random.default_rng(seed)
    R = 6 if seed % 2 else 4
    K = 256 if seed < 4 else 1024
    pool = _random_masks(rng, 5000, R, 0.15 + 0.05 * seed)
    boxes = rng.random((5000, 6)).astype(np.float32)
    boxes[:, 3:] += boxes[:, :3]
    cb = oracle.codebook(pool, boxes, R, K)
    queries = _random_masks(rng, 3000, R, 0.05 + 0.03 * seed)
    req = oracle.req_luts(cb, R)
    a = oracle.alg3(queries, req, K, R)
    b = oracle.naive_search(queries, cb, R)
    assert (a == b).all()
    assert _is_superset(cb[a], queries).all()
    # tightest: no superset entry has fewer bits
    pcs = popcount64(cb)
    for q, i in zip(queries[:200], a[:200]):
        sup = _is_superset(cb, q[None, :])
        assert pcs[i] == pcs[sup].min()


def _scene_masks(name, R, small_oracle):
    if name == "small":
        return small_oracle[f"masks{R}"], small_oracle["bvh"].slot_boxes()
    tris = scenes.segment_rows(0) if name == "segments" else scenes.lattice_copies(40)
    bvh = oracle.bvh_build(tris)
    _, delta = oracle.default_bounds(tris)
    return oracle.object_masks(tris, bvh, R, delta), bvh.slot_boxes()


@pytest.mark.parametrize("name,R,K", [("small", 6, 256), ("small", 4, 64), ("segments", 6, 64),
                                      ("segments", 4, 64), ("lattice40", 6, 64), ("lattice40", 4, 64)])
def test_codebook_structure_and_importance(small_oracle, name, R, K):
    """Ranking recomputed from its definition. Segment rows: at R = 4 and K = 64 the last chosen
    place falls among three distinct masks tied at importance 0, so the value order decides it;
    the lattice has more distinct masks than K - 1."""
    masks, boxes = _scene_masks(name, R, small_oracle)
    cb = oracle.codebook(masks, boxes, R, K)
    full = _full(R)
    assert (cb == full).all(axis=1).any()
    pcs = popcount64(cb)
    assert (np.diff(pcs) >= 0).all()
    # importance per distinct pattern, recomputed in float64 (sums in slot order)
    d = boxes[:, 3:].astype(np.float64) - boxes[:, :3].astype(np.float64)
    sa = 2.0 * ((d[:, 0] * d[:, 1] + d[:, 1] * d[:, 2]) + d[:, 2] * d[:, 0])
    imp = sa * popcount64(masks) / R ** 3
    acc = {}
    for s in range(masks.shape[0]):
        k = masks[s].tobytes()
        acc[k] = acc.get(k, 0.0) + imp[s]
    acc.pop(full.tobytes(), None)
    ranked = sorted(acc.items(), key=lambda kv: (-kv[1], kv[0][::-1]))
    want = {k for k, _ in ranked[:K - 1]}
    got = {row.tobytes() for row in cb if not (row == full).all()}
    if len(acc) >= K - 1:
        assert got == want
    else:
        assert got == set(acc)
    # padding: the full mask fills every entry the chosen patterns leave
    assert int((cb == full).all(axis=1).sum()) == K - min(len(acc), K - 1)


def test_paper_layout_facts():
    """Sizes the paper states (Sect. 3.2.4, 4.4): mask bytes and compression rates."""
    with open(GOLDEN) as f:
        facts = json.load(f)
    for R, nbytes in facts["mask_bytes"].items():
        assert int(R) ** 3 / 8 == nbytes
    for R, rate in facts["compression_rate_k256"].items():
        # one byte of index replaces R^3/8 bytes of mask
        assert int(R) ** 3 / 8 == rate
    bvh4 = facts["bvh4_node_bytes_R4"]
    box, ref, mask, index = 24, 4, 8, 1
    assert 4 * box + 4 * ref == bvh4["plain"]
    assert bvh4["plain"] + 4 * mask == bvh4["uncompressed"]
    assert bvh4["plain"] + 4 * index == bvh4["compressed"]
    for R, n in facts["requirement_tables_b8"].items():
        assert -(-int(R) ** 3 // 8) == n
