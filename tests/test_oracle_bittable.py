"""Pins of the oracle's 2-D bit table (Sect. 3.2.2): properties that follow
from the definition bit (key, k) = (ray mask AND codebook entry k) != 0.

* the full codebook entry answers 1 for every ray mask (a ray mask is never
  empty);
* a ray that enters and leaves in the same cell has that single cell as its
  ray mask (strict overlap), so it answers 1 exactly for the entries with that
  voxel set, computed here from voxel coordinates;
* supersets answer at least as often as their subsets (monotone);
* an all-zero entry never answers 1.
"""
import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("R", [4, 6])
def test_bit_table_properties(small_oracle, R):
    bvh = small_oracle["bvh"]
    cb, _ = oracle.compress(small_oracle[f"masks{R}"], bvh.slot_boxes(), R, 256)
    cb = cb.copy()
    cb[0] = 0  # plant an empty entry (the codebook itself never has one)
    T = oracle.bit_table(R, cb)
    K = cb.shape[0]
    bits = np.unpackbits(T.view(np.uint8), axis=1, bitorder="little")[:, :K].astype(bool)
    pc = np.unpackbits(cb.view(np.uint8), axis=1).sum(1)
    full = int(np.flatnonzero(pc == R ** 3)[0])
    assert bits[:, full].all()
    assert not bits[:, 0].any()
    cbits = oracle.mask_bits(cb, R).astype(bool)  # [K, R^3]
    coords = np.array([(x, y, z) for z in range(R) for y in range(R) for x in range(R)])
    for (x, y, z) in [(0, 0, 0), (R - 1, 1, 2), (2, R - 1, R - 1), (1, 1, 1)]:
        key = ((((x * R + y) * R + z) * R + x) * R + y) * R + z
        near = (coords == np.array([x, y, z])).all(1)
        want = (cbits[:, near]).any(1)
        assert (bits[key] == want).all()
    # monotone: an entry that contains another answers 1 wherever the other does
    rng = np.random.default_rng(R)
    for _ in range(200):
        i, j = rng.integers(1, K, 2)
        if ((cb[i] & ~cb[j]) == 0).all():  # cb[j] contains cb[i]
            assert (bits[:, j] >= bits[:, i]).all()


@pytest.mark.parametrize("R", [4, 6])
def test_bit_table_rows_symmetric_in_entry_and_exit(small_oracle, R):
    """Row (b, e) equals row (e, b): the traversal looks up the ordered pair only."""
    lut = small_oracle[f"lut{R}"]
    rng = np.random.default_rng(R)
    cb = np.unique(rng.integers(0, 2 ** 63, size=(256, oracle.words_for(R)), dtype=np.int64).astype(np.uint64),
                   axis=0)[:128]
    table = oracle.bit_table(R, cb, lut)
    c3 = R ** 3
    key = np.arange(R ** 6)
    b, e = key // c3, key % c3
    assert (table[key] == table[e * c3 + b]).all()
