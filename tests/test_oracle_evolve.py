"""Pins for the generation-step reference (oracle/evolve_ref.py): its hash
against the published SplitMix64 stream, the closed-form properties of SBX
and polynomial mutation, and the objective map's radius law."""
import math
import os

import numpy as np

from oracle import evolve_ref as ev

GOLD = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed0.txt")
GAMMA = 0x9E3779B97F4A7C15


def test_splitmix64_published_stream():
    vals = [int(s, 16) for s in open(GOLD).read().split("\n") if s.startswith("0x")]
    for i, v in enumerate(vals):
        assert ev.splitmix64((i * GAMMA) & ev.MASK64) == v


def test_hash_fields_are_disjoint():
    # every field changes the hash; fields do not overlap inside the counter
    base = ev.h(7, 3, ev.TAG_SBX, 11, 5)
    assert ev.h(8, 3, ev.TAG_SBX, 11, 5) != base
    assert ev.h(7, 4, ev.TAG_SBX, 11, 5) != base
    assert ev.h(7, 3, ev.TAG_PA, 11, 5) != base
    assert ev.h(7, 3, ev.TAG_SBX, 12, 5) != base
    assert ev.h(7, 3, ev.TAG_SBX, 11, 6) != base
    hs = {ev.h(1, g, t, i, j) for g in range(3) for t in (4, 5) for i in range(50) for j in range(12)}
    assert len(hs) == 3 * 2 * 50 * 12


def test_u01_grid():
    assert ev.u01(0) == 0.0
    assert ev.u01(ev.MASK64) == 1.0 - 2.0 ** -24
    # exactly representable in float32
    for x in (ev.h(3, 1, 7, i, 0) for i in range(100)):
        u = ev.u01(x)
        assert float(np.float32(u)) == u


def test_sbx_properties():
    # beta(1/2) = 1: children equal their parents; children are symmetric about
    # the parents' mean; spread factor |c1 - c2| / |x1 - x2| = beta
    assert ev.sbx_beta(0.5) == 1.0
    assert ev.sbx_beta(0.0) == 0.0
    x1, x2 = 0.3, 0.7
    for u in (0.01, 0.2, 0.5, 0.8, 0.99):
        b = ev.sbx_beta(u)
        c1 = 0.5 * ((1 + b) * x1 + (1 - b) * x2)
        c2 = 0.5 * ((1 - b) * x1 + (1 + b) * x2)
        assert abs((c1 + c2) - (x1 + x2)) < 1e-15
        assert abs(abs(c1 - c2) / abs(x1 - x2) - b) < 1e-12
    # the spread factor's density is 0.5 (eta+1) beta^eta below 1: P(beta <= b)
    # = 0.5 b^(eta+1), i.e. beta(u) inverts that CDF
    for b in (0.3, 0.9, 1.0):
        u = 0.5 * b ** (ev.ETA_C + 1)
        assert abs(ev.sbx_beta(u) - b) < 1e-12
    # above 1: P(beta > b) = 0.5 b^-(eta+1)
    for b in (1.1, 2.0):
        u = 1 - 0.5 * b ** -(ev.ETA_C + 1)
        assert abs(ev.sbx_beta(u) - b) < 1e-9


def test_polynomial_mutation_properties():
    assert ev.pm_delta(0.5) == 0.0
    assert ev.pm_delta(0.0) == -1.0
    assert abs(ev.pm_delta(1.0 - 2 ** -24) - 1.0) < 0.5
    us = np.linspace(0.0, 1.0 - 2 ** -24, 1001)
    ds = [ev.pm_delta(u) for u in us]
    assert all(b >= a for a, b in zip(ds, ds[1:]))
    # antisymmetry about u = 1/2
    for u in (0.1, 0.3, 0.45):
        assert abs(ev.pm_delta(u) + ev.pm_delta(1 - u)) < 1e-12


def test_objective_map_radius_and_direction():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((4, 11))
    X = rng.random((500, 12))
    F = ev.objectives(X, A)
    assert np.all(F >= 0)
    rad = np.linalg.norm(F, axis=1)
    assert np.allclose(rad, 1 - 0.3 * np.log(1 - X[:, -1]), rtol=1e-12)
    # direction: proportional to |A (x - 1/2)|
    y = np.abs((X[:, :-1] - 0.5) @ A.T)
    assert np.allclose(F / rad[:, None], y / np.linalg.norm(y, axis=1, keepdims=True))
    # at the centre the direction is the diagonal
    Xc = np.full((1, 12), 0.5)
    Fc = ev.objectives(Xc, A)
    assert np.allclose(Fc, np.full(4, 1 / 2.0) * 1.0 * (1 - 0.3 * math.log(0.5)))


def test_objective_map_radius_law():
    # at uniform x the radius is 1 + Exponential(mean 0.3)
    rng = np.random.default_rng(1)
    X = rng.random((20000, 12))
    F = ev.objectives(X, rng.standard_normal((3, 11)))
    g = np.linalg.norm(F, axis=1) - 1
    assert abs(g.mean() - 0.3) < 0.01
    assert abs(np.median(g) - 0.3 * math.log(2)) < 0.01


def test_offspring_shapes_and_bounds():
    P = ev.init_population(40, 12, 5)
    assert P.shape == (40, 12) and np.all((P >= 0) & (P < 1))
    O = ev.offspring(P, 5, 1)
    assert O.shape == (40, 12) and np.all((O >= 0) & (O <= ev.XMAX))
    # each offspring pair without mutation is the SBX pair of its parents
    k = 3
    a = ev.h(5, 1, ev.TAG_PA, k, 0) % 40
    b = ev.h(5, 1, ev.TAG_PB, k, 0) % 40
    for j in range(12):
        m0 = ev.u01(ev.h(5, 1, ev.TAG_PM_APPLY, 2 * k, j)) < ev.pm_threshold(12)
        m1 = ev.u01(ev.h(5, 1, ev.TAG_PM_APPLY, 2 * k + 1, j)) < ev.pm_threshold(12)
        c1, c2 = O[2 * k, j], O[2 * k + 1, j]
        if m0 or m1 or not (0 < c1 < ev.XMAX and 0 < c2 < ev.XMAX):
            continue
        x1, x2 = P[a, j], P[b, j]
        assert abs((c1 + c2) - (x1 + x2)) < 1e-12
        beta = ev.sbx_beta(ev.u01(ev.h(5, 1, ev.TAG_SBX, k, j)))
        assert abs(abs(c1 - c2) - beta * abs(x1 - x2)) < 1e-12
