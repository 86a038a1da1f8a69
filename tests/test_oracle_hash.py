"""Pins for the SplitMix64 tie-break key used by the oracle."""
import os

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed0.txt")
GAMMA = 0x9E3779B97F4A7C15
MASK = 2**64 - 1


def test_published_stream():
    vals = [int(s, 16) for s in open(GOLD).read().split("\n") if s.startswith("0x")]
    assert len(vals) == 3
    for i, v in enumerate(vals):
        assert oracle.splitmix64((i * GAMMA) & MASK) == v


def test_key_is_injective_in_ref():
    # sm64 is a bijection of 64-bit words, so keys of distinct refs at one level differ
    ks = {oracle.key(12345, 1, j, 7) for j in range(20000)}
    assert len(ks) == 20000


def test_key_depends_on_every_field():
    base = oracle.key(1, 1, 5, 3)
    assert oracle.key(2, 1, 5, 3) != base
    assert oracle.key(1, 2, 5, 3) != base
    assert oracle.key(1, 1, 6, 3) != base
    assert oracle.key(1, 1, 5, 4) != base


def test_key_low_bits_uniform():
    # chi-square of key mod 7 over 70000 refs: uniform picks among 7 members
    counts = [0] * 7
    for j in range(70000):
        counts[oracle.key(99, 2, j, 1) % 7] += 1
    chi2 = sum((c - 10000) ** 2 / 10000 for c in counts)
    assert chi2 < 22.5  # 6 dof, p = 0.001
