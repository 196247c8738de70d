"""Pins of the oracle's ray-mask LUT (Sect. 3.1.1, Alg. 1).

The LUT entry (beg, end) must be the union of grid cells crossed by straight
segments that start anywhere in cell ``beg`` and end anywhere in cell
``end`` (the sweep of Sect. 3.1.1 covers "all possible rays" between the two
cells). Pinned by closed forms, by sampling segments in float64 (nothing
crossed may be missing) and by explicit witness segments (nothing set may be
spurious).
"""
import itertools

import numpy as np
import pytest

import oracle


def _cells(R):
    return [np.array(c) for c in itertools.product(range(R), repeat=3)]  # (x, y, z)


def _key(R, b, e):
    # key order: beg x, y, z then end x, y, z, most significant first
    k = 0
    for v in (*b, *e):
        k = k * R + int(v)
    return k


def _bit(R, c):
    return int(c[0]) + R * int(c[1]) + R * R * int(c[2])


@pytest.fixture(scope="module", params=[4, 6])
def lut(request):
    R = request.param
    return R, oracle.mask_bits(oracle.raymask_lut(R), R)


def test_shape_and_sizes(lut):
    R, bits = lut
    # six-dimensional table (Sect. 3.1.1): R^6 keys of R^3 bits
    assert bits.shape == (R ** 6, R ** 3)


def test_same_cell_is_single_voxel(lut):
    R, bits = lut
    for c in _cells(R):
        row = bits[_key(R, c, c)]
        assert row.sum() == 1 and row[_bit(R, c)]


def test_axis_aligned_runs(lut):
    R, bits = lut
    rng = np.random.default_rng(3)
    for _ in range(200):
        b = rng.integers(0, R, 3)
        e = b.copy()
        ax = rng.integers(0, 3)
        e[ax] = rng.integers(0, R)
        row = bits[_key(R, b, e)]
        lo, hi = min(b[ax], e[ax]), max(b[ax], e[ax])
        expect = np.zeros(R ** 3, bool)
        for v in range(lo, hi + 1):
            c = b.copy()
            c[ax] = v
            expect[_bit(R, c)] = True
        assert (row == expect).all(), (b, e)


def test_symmetry_and_bounds(lut):
    R, bits = lut
    rng = np.random.default_rng(4)
    for _ in range(500):
        b, e = rng.integers(0, R, 3), rng.integers(0, R, 3)
        row = bits[_key(R, b, e)]
        assert (row == bits[_key(R, e, b)]).all()
        assert row[_bit(R, b)] and row[_bit(R, e)]
        lo, hi = np.minimum(b, e), np.maximum(b, e)
        for c in _cells(R):
            if row[_bit(R, c)]:
                assert (c >= lo).all() and (c <= hi).all()


def test_diagonal_step_is_2x2_square(lut):
    R, bits = lut
    row = bits[_key(R, (0, 0, 0), (1, 1, 0))]
    expect = {_bit(R, c) for c in [(0, 0, 0), (1, 0, 0), (0, 1, 0), (1, 1, 0)]}
    assert set(np.flatnonzero(row)) == expect


def test_sampled_segments_are_covered(lut):
    """Every cell crossed by a sampled segment between the two cells is set."""
    R, bits = lut
    rng = np.random.default_rng(5)
    n_keys, n_seg, n_s = 3000, 16, 201
    b = rng.integers(0, R, (n_keys, 3))
    e = rng.integers(0, R, (n_keys, 3))
    keys = np.array([_key(R, x, y) for x, y in zip(b, e)])
    p = b[:, None, :] + rng.random((n_keys, n_seg, 3))
    q = e[:, None, :] + rng.random((n_keys, n_seg, 3))
    s = np.linspace(0.0, 1.0, n_s)
    x = p[:, :, None, :] + s[None, None, :, None] * (q - p)[:, :, None, :]
    cell = np.floor(x).astype(np.int64)
    cell = np.minimum(cell, R - 1)
    flat = cell[..., 0] + R * cell[..., 1] + R * R * cell[..., 2]
    ok = np.take_along_axis(bits[keys], flat.reshape(n_keys, -1), axis=1)
    assert ok.all()


def test_witness_for_every_set_bit(lut):
    """Each set voxel is crossed by an explicit segment between the two cells.

    From the sweep condition there is an s* with |beg + s*(end-beg) - v| < 1 on
    every axis; the offset f chosen inside both [0,1) and v - (beg + s*D) +
    [0,1) puts beg+f in cell beg, end+f in cell end, and the point at s* in v.
    """
    R, bits = lut
    rng = np.random.default_rng(6)
    keys = rng.integers(0, R ** 6, 1500)
    for k in keys:
        digits = [(k // R ** (5 - i)) % R for i in range(6)]
        b, e = np.array(digits[:3], float), np.array(digits[3:], float)
        D = e - b
        for vb in np.flatnonzero(bits[k]):
            v = np.array([vb % R, (vb // R) % R, vb // (R * R)], float)
            lo, hi = 0.0, 1.0
            for i in range(3):
                if D[i] == 0:
                    assert v[i] == b[i]
                    continue
                a0, a1 = (v[i] - 1 - b[i]) / D[i], (v[i] + 1 - b[i]) / D[i]
                a0, a1 = min(a0, a1), max(a0, a1)
                lo, hi = max(lo, a0), min(hi, a1)
            assert lo < hi or (lo == hi and 0.0 <= lo <= 1.0)
            s = 0.5 * (lo + hi)
            c = b + s * D
            flo = np.maximum(0.0, v - c)
            fhi = np.minimum(1.0, v + 1 - c)
            assert (flo < fhi).all()
            f = 0.5 * (flo + fhi)
            pt = c + f
            assert (np.floor(pt) == v).all()
            assert (np.floor(b + f) == b).all() and (np.floor(e + f) == e).all()
