"""Pins for the reference quality indicators (oracle/quality_ref.py): closed
forms of IGD for scaled fronts, brute force on tiny inputs, the published
SplitMix64 stream for the sample generator, and exact box volumes for the
hypervolume count."""
import itertools
import math
import os

import numpy as np

from oracle import quality_ref as q

GOLD = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed0.txt")
GAMMA = 0x9E3779B97F4A7C15
MASK = 2**64 - 1


def unit_front(m, p):
    """Unit vectors along the compositions of p into m parts."""
    rows = [c for c in itertools.product(range(p + 1), repeat=m) if sum(c) == p]
    R = np.array(rows, np.float64)
    return R / np.linalg.norm(R, axis=1, keepdims=True)


def test_igd_of_the_front_itself_is_zero():
    R = unit_front(3, 6)
    assert q.igd(R, R) == 0.0


def test_igd_of_a_scaled_front_is_the_scale_gap():
    # for unit r and s: ||r - c s||^2 = 1 + c^2 - 2c cos >= (1 - c)^2, with
    # equality at s = r, so every distance is |1 - c|
    R = unit_front(4, 5)
    for c in (0.5, 0.9, 1.0, 1.25, 1.5):
        assert abs(q.igd(c * R, R) - abs(1 - c)) < 1e-12


def test_igd_brute_force():
    rng = np.random.default_rng(3)
    F = rng.random((23, 3))
    R = rng.random((11, 3))
    want = sum(min(math.sqrt(sum((r[k] - f[k]) ** 2 for k in range(3))) for f in F)
               for r in R) / len(R)
    assert abs(q.igd(F, R) - want) < 1e-12


def test_sample_generator_follows_splitmix64():
    vals = [int(s, 16) for s in open(GOLD).read().split("\n") if s.startswith("0x")]
    for i, v in enumerate(vals):
        assert int(q.splitmix64(np.uint64((i * GAMMA) & MASK))) == v
    # sample (i, k) of a unit box is (sm64(seed ^ sm64(i << 8 | k)) >> 40) * 2^-24
    y = q.hv_samples([0, 0], [1, 1], 3, seed=77)
    for i in range(3):
        for k in range(2):
            inner = int(q.splitmix64(np.uint64((i << 8) | k)))
            h = int(q.splitmix64(np.uint64(77 ^ inner)))
            assert y[i, k] == np.float32((h >> 40) / 2**24)


def test_samples_stay_in_the_box():
    ideal = np.array([0.1, -2.0, 3.0], np.float32)
    ref = np.array([0.3, 5.0, 3.0], np.float32)
    y = q.hv_samples(ideal, ref, 5000, seed=5)
    assert np.all(y >= ideal) and np.all(y <= ref)
    assert np.all(y[:, 2] == 3.0)


def test_hv_count_brute_force():
    rng = np.random.default_rng(4)
    F = rng.random((7, 3)).astype(np.float32)
    ideal, ref = np.zeros(3, np.float32), np.ones(3, np.float32)
    y = q.hv_samples(ideal, ref, 300, seed=9)
    want = sum(any(all(f[k] <= s[k] for k in range(3)) for f in F) for s in y)
    assert q.hv_count(F, ideal, ref, 300, 9) == want


def test_hv_of_one_point_and_of_two_boxes():
    # one point p: the dominated part of the box is [max(p, ideal), ref]
    ideal, ref = np.zeros(3, np.float32), np.ones(3, np.float32)
    S = 200000
    p = np.array([[0.25, 0.5, 0.75]], np.float32)
    frac = q.hv_count(p, ideal, ref, S, 1) / S
    exact = 0.75 * 0.5 * 0.25
    assert abs(frac - exact) < 5 * math.sqrt(exact * (1 - exact) / S)
    # two points: inclusion-exclusion of their boxes
    P = np.array([[0.25, 0.5, 0.75], [0.5, 0.25, 0.5]], np.float32)
    exact2 = 0.75 * 0.5 * 0.25 + 0.5 * 0.75 * 0.5 - 0.5 * 0.5 * 0.25
    frac2 = q.hv_count(P, ideal, ref, S, 2) / S
    assert abs(frac2 - exact2) < 5 * math.sqrt(exact2 * (1 - exact2) / S)


def test_hv_box_is_the_papers():
    ideal, ref = q.hv_box([1.0, 2.0], [3.0, 4.0])
    assert np.allclose(ideal, [0.9, 1.8]) and np.allclose(ref, [3.03, 4.04])
