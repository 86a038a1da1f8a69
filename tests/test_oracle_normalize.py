"""Pins for the oracle's normalization (Algorithm 1/2 "Normalize"; Deb & Jain
2014 procedure): closed forms, a library solve, exact scaling, degeneracy."""
import numpy as np
import pytest

import oracle
from paper_2504_06067_amd import workloads as wl


def all_st(M):
    return np.zeros(M, np.int32), np.array([0, 0, M, 1], np.int32)


@pytest.mark.parametrize("m", [2, 3, 5, 10, 32, 128, 512])
def test_axis_points_give_identity(m):
    # unit axis points present, everything else >= 0.01 in every objective:
    # ideal 0, extremes are the axis points, intercepts 1, Fn == F
    rng = np.random.default_rng(m)
    F = np.concatenate([np.eye(m), 0.01 + rng.random((50, m))]).astype(np.float32)
    rank, fi = all_st(len(F))
    r = oracle.normalize(F, rank, fi)
    assert np.array_equal(r["ideal"], np.zeros(m))
    assert list(r["extreme"]) == list(range(m))
    assert r["degenerate"] == 0
    assert np.array_equal(r["intercept"], np.ones(m))
    assert np.array_equal(r["Fn"], F.astype(np.float64))


def test_two_objectives_closed_form():
    # m = 2: the extreme for axis 1 is the point of least f2 (and vice versa),
    # so the intercepts are the translated far coordinates of those points
    rng = np.random.default_rng(7)
    for _ in range(20):
        F = (1.0 + rng.random((40, 2))).astype(np.float32)
        rank, fi = all_st(40)
        r = oracle.normalize(F, rank, fi)
        z = F.astype(np.float64).min(axis=0)
        e1 = int(np.lexsort((np.arange(40), F[:, 0], F[:, 1]))[0])  # least f2, then f1
        e2 = int(np.lexsort((np.arange(40), F[:, 1], F[:, 0]))[0])
        assert r["extreme"][0] == e1 and r["extreme"][1] == e2
        a = np.array([F[e1, 0] - z[0], F[e2, 1] - z[1]], np.float64)
        assert r["degenerate"] == 0
        np.testing.assert_allclose(r["intercept"], a, rtol=1e-14)


@pytest.mark.parametrize("m", [3, 6, 10])
def test_intercepts_match_library_solve(m):
    rng = np.random.default_rng(m)
    F = wl.objectives(rng, 400, m, "exp")
    rank, fi = all_st(400)
    r = oracle.normalize(F, rank, fi)
    z = F.astype(np.float64).min(axis=0)
    E = F[r["extreme"]].astype(np.float64) - z
    b = np.linalg.solve(E, np.ones(m))
    assert r["degenerate"] == 0
    np.testing.assert_allclose(1.0 / r["intercept"], b, rtol=1e-10)
    np.testing.assert_allclose(r["Fn"], (F - z) / r["intercept"], rtol=1e-12)


def test_power_of_two_scaling_is_exact():
    inst = wl.plain_instance("large", 2, M=2000)
    rank, fi = oracle.nd_sort(inst["F"], 1000)
    r1 = oracle.normalize(inst["F"], rank, fi)
    r2 = oracle.normalize(inst["F"] * np.float32(8.0), rank, fi)
    assert np.array_equal(r2["ideal"], 8.0 * r1["ideal"])
    assert np.array_equal(r2["extreme"], r1["extreme"])
    assert np.array_equal(r2["intercept"], 8.0 * r1["intercept"])
    st = rank <= fi[0]
    assert np.array_equal(r2["Fn"][st], r1["Fn"][st])


def test_degenerate_falls_back_to_max():
    # objectives 2 and 3 identical: the extreme rows are linearly dependent
    rng = np.random.default_rng(3)
    x = rng.random((60, 2))
    F = np.stack([x[:, 0], x[:, 1], x[:, 1]], axis=1).astype(np.float32)
    rank, fi = all_st(60)
    r = oracle.normalize(F, rank, fi)
    z = F.astype(np.float64).min(axis=0)
    assert r["degenerate"] == 1
    np.testing.assert_array_equal(r["intercept"], F.astype(np.float64).max(axis=0) - z)


def test_only_st_rows_count():
    # points outside S_t must not move the ideal point or the extremes
    rng = np.random.default_rng(4)
    F = (1 + rng.random((30, 3))).astype(np.float32)
    rank = np.zeros(30, np.int32)
    rank[20:] = oracle.UNRANKED
    F[25] = 0.0  # would be the ideal if it counted
    fi = np.array([0, 0, 10, 1], np.int32)
    r = oracle.normalize(F, rank, fi)
    np.testing.assert_array_equal(r["ideal"], F[:20].astype(np.float64).min(axis=0))
    assert np.all(r["extreme"] < 20)
    assert np.all(np.isnan(r["Fn"][20:]))


# Hand-built extreme sets (dyadic values, so every translated objective and
# every 1e6 multiple below is exact in float32 and float64; ideal point 0).
# Axis points e1 = (1, 0, 0) and e2 = (0, 1, 0) fix b_1 = b_2 = 1; the third
# row decides b_3 of the hyperplane f . b = 1 through the extreme points.
def three_extremes(e3, extra=()):
    rows = [(1.0, 0.0, 0.0), (0.0, 1.0, 0.0), e3, *extra]
    return np.array(rows, np.float32)


def test_asf_tie_goes_to_least_index():
    # Two points whose axis-1 ASF is the same product 1e6 * 2^-10 (their first
    # objectives differ and stay below it): the least index is the extreme,
    # in either order of the two (a "last index" rule, or an ASF without the
    # 1e6 factor, picks index 4 in one of the orders).
    t = 2.0 ** -10
    base = [(1.0, 1.0, 1.0), (0.0, 1.0, 0.5), (0.75, 0.0, 1.0)]
    for lo, hi in ((0.5, 0.25), (0.25, 0.5)):
        F = np.array(base + [(lo, t, 0.0), (hi, t, 0.0)], np.float32)
        rank, fi = all_st(len(F))
        r = oracle.normalize(F, rank, fi)
        assert np.array_equal(r["ideal"], np.zeros(3))
        assert r["extreme"][0] == 3, (lo, hi, r["extreme"])


def test_negative_intercept_is_degenerate():
    # e3 = (7/8, 7/8, 1/8): ASF_3 = 875000 < 1e6, so it is the axis-3 extreme;
    # the plane through the three rows has b_3 = (1 - 7/4) / (1/8) = -6 <= 0
    F = three_extremes((0.875, 0.875, 0.125))
    r = oracle.normalize(F, *all_st(3))
    assert list(r["extreme"]) == [0, 1, 2]
    z = np.zeros(3)
    E = F.astype(np.float64) - z
    b = np.linalg.solve(E, np.ones(3))
    assert b[2] == -6.0  # the branch is reached by a solvable, non-singular system
    assert r["degenerate"] == 1
    assert np.array_equal(r["intercept"], np.array([1.0, 1.0, 0.125]))


def test_zero_b_is_degenerate():
    # e3 = (1/2, 1/2, 1/8) lies on f1 + f2 = 1: b_3 = 0 exactly (a_3 infinite)
    F = three_extremes((0.5, 0.5, 0.125))
    r = oracle.normalize(F, *all_st(3))
    assert list(r["extreme"]) == [0, 1, 2]
    assert r["degenerate"] == 1
    assert np.array_equal(r["intercept"], np.array([1.0, 1.0, 0.125]))


@pytest.mark.parametrize("far,degen", [(4.0, 1), (1.0, 0)])
def test_tiny_intercept_relative_to_span(far, degen):
    # e3 = (1/4, 1/4, 2^-20) gives b_3 = (1 - 1/2) / 2^-20, i.e. a_3 = 2^-19
    # (about 1.9e-6). A fourth point (2, 2, far) sets max f'_3 = far without
    # being an extreme (its ASF values are 2e6 or more). The intercept is
    # rejected iff a_3 < 1e-6 * far: relative, so far = 4 rejects it and
    # far = 1 keeps it (an absolute 1e-6 threshold would keep both).
    c = 2.0 ** -20
    F = three_extremes((0.25, 0.25, c), extra=[(2.0, 2.0, far)])
    r = oracle.normalize(F, *all_st(4))
    assert list(r["extreme"]) == [0, 1, 2]
    assert r["degenerate"] == degen
    if degen:
        assert np.array_equal(r["intercept"], np.array([2.0, 2.0, far]))
    else:
        assert np.array_equal(r["intercept"], np.array([1.0, 1.0, 2.0 ** -19]))


@pytest.mark.parametrize("m", [32, 64, 200])
def test_many_objective_intercepts_match_library_solve(m):
    # extreme rows near the axes (axis k at 1 + u_k, off-axis values below
    # 1e-7, so that 1e6 times them stays below 1) plus far points: the
    # oracle's extremes are those rows and its intercepts solve the same
    # system as numpy's LU
    rng = np.random.default_rng(m)
    E = 1e-7 * rng.random((m, m)) + np.diag(1.0 + rng.random(m))
    zero_rest = np.zeros(m)
    zero_rest[0] = 3.0            # objectives 2..m reach 0 here (ASF_1 = 3)
    zero_first = np.full(m, 3.0)
    zero_first[0] = 0.0           # objective 1 reaches 0 here
    far = 0.5 + rng.random((40, m))
    F = np.concatenate([E, [zero_rest, zero_first], far]).astype(np.float32)
    rank, fi = all_st(len(F))
    r = oracle.normalize(F, rank, fi)
    assert np.array_equal(r["ideal"], np.zeros(m))
    assert list(r["extreme"]) == list(range(m))
    b = np.linalg.solve(F[:m].astype(np.float64), np.ones(m))
    assert r["degenerate"] == 0
    np.testing.assert_allclose(1.0 / r["intercept"], b, rtol=1e-10)
