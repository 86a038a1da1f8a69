"""The parallel decode of a reference's random picks, checked against the
serial process on the CPU.

In the niche step a reference with c candidates (ascending index order) makes
t picks; pick p takes the candidate of rank k_p among those still remaining
(the nearest candidate's position for a first pick at niche count 0, else
key mod (c - p)). The pick kernel computes every k_p up front and decodes the
positions in parallel: pick i's position is k_i, raised by one for each
earlier pick j (taken from i - 1 down to 0) whose rank is at most the running
value. This test checks that rule against the serial remove-and-select
process on random rank sequences, including repeated ranks and t = c.
"""
import numpy as np
import pytest


def serial(c, ranks):
    remaining = list(range(c))
    out = []
    for k in ranks:
        out.append(remaining.pop(k))
    return out


def decode(ranks):
    out = []
    for i, r in enumerate(ranks):
        for j in range(i - 1, -1, -1):
            if ranks[j] <= r:
                r += 1
        out.append(r)
    return out


@pytest.mark.parametrize("seed", range(40))
def test_decode_equals_serial(seed):
    rng = np.random.default_rng(seed)
    c = int(rng.integers(1, 300))
    t = int(rng.integers(1, c + 1))
    # rank of pick p is uniform over the c - p remaining candidates; small
    # ranges make repeated ranks (and runs of zeros) common
    ranks = [int(rng.integers(0, c - p)) if seed % 3 else int(rng.integers(0, min(3, c - p)))
             for p in range(t)]
    assert decode(ranks) == serial(c, ranks)


def test_decode_worked_cases():
    # a naive forward update (shift later ranks past each removal) fails the
    # first case; the backward re-insertion does not
    assert serial(5, [2, 1, 1]) == decode([2, 1, 1]) == [2, 1, 3]
    assert serial(5, [0, 0, 0]) == decode([0, 0, 0]) == [0, 1, 2]
    assert serial(4, [1, 0, 1]) == decode([1, 0, 1]) == [1, 0, 3]
    assert serial(6, [5, 4, 3, 2, 1, 0]) == decode([5, 4, 3, 2, 1, 0]) == [5, 4, 3, 2, 1, 0]
