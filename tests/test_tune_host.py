"""Autotuner candidate set (host logic, no GPU): every compiled (block, stack)
pair with each chunk, partition count, wave cap and sort choice; the codebook
placement only for LUT-mode scenes, where it is the one extra dimension;
every shape with each leaf- and refill-gathering threshold."""
from paper_2305_08343_amd import tune


def test_candidates_cover_the_grid_once():
    plain, lut = tune.candidates(), tune.candidates(lut=True)
    n = (len(tune.PAIRS) * len(tune.CHUNKS) * len(tune.PARTS) * len(tune.WAVES) * len(tune.SORT)
         * len(tune.GATHER) * len(tune.REFILL))
    assert len(plain) == n and len(set(plain)) == n
    assert len(lut) == 2 * n and len(set(lut)) == 2 * n
    assert all(len(c) == 9 and c[6] == 0 for c in plain)
    assert {c[6] for c in lut} == {0, 1}
    assert {c[7] for c in plain} == set(tune.GATHER) and 0 in tune.GATHER
    assert {c[8] for c in plain} == set(tune.REFILL) and 1 in tune.REFILL
    assert {c[:6] + c[7:] for c in lut} == {c[:6] + c[7:] for c in plain}
    assert all((c[0], c[1]) in tune.PAIRS for c in lut)
