"""Pins for the oracle's association (Sec. II-C, Eq. 1 read as the true
perpendicular distance, Algorithm 2 argmin/min)."""
import numpy as np
import pytest

import oracle
from paper_2504_06067_amd import workloads as wl


def all_st(M):
    return np.zeros(M, np.int32), np.array([0, 0, M, 1], np.int32)


@pytest.mark.parametrize("m,p", [(2, 9), (3, 12), (5, 6), (10, 3), (32, 2), (128, 1), (512, 1)])
def test_points_on_reference_directions(m, p):
    Z = wl.das_dennis(m, p)
    H = len(Z)
    rng = np.random.default_rng(m)
    c = rng.uniform(0.5, 2.0, H)
    Fn = Z.astype(np.float64) * c[:, None]
    rank, fi = all_st(H)
    pi, d = oracle.associate(Fn, rank, fi, Z)
    assert np.array_equal(pi, np.arange(H))
    assert np.all(d < 1e-12)


def test_two_d_cross_product():
    rng = np.random.default_rng(0)
    Z = wl.das_dennis(2, 7).astype(np.float64)
    Fn = rng.random((200, 2))
    rank, fi = all_st(200)
    pi, d = oracle.associate(Fn, rank, fi, Z.astype(np.float32))
    W = Z / np.linalg.norm(Z, axis=1, keepdims=True)
    cross = np.abs(Fn[:, None, 0] * W[None, :, 1] - Fn[:, None, 1] * W[None, :, 0])
    np.testing.assert_allclose(d, cross.min(axis=1), rtol=1e-12, atol=1e-15)
    best = cross.min(axis=1, keepdims=True)
    # chosen reference is within rounding of the cross-product minimum
    chosen = cross[np.arange(200), pi]
    np.testing.assert_allclose(chosen, best[:, 0], rtol=1e-12, atol=1e-15)


def test_three_d_cross_product():
    rng = np.random.default_rng(1)
    Z = wl.das_dennis(3, 10).astype(np.float64)
    Fn = rng.random((300, 3)) * 2
    rank, fi = all_st(300)
    pi, d = oracle.associate(Fn, rank, fi, Z.astype(np.float32))
    W = Z / np.linalg.norm(Z, axis=1, keepdims=True)
    cr = np.linalg.norm(np.cross(Fn[:, None, :], W[None, :, :]), axis=2)
    np.testing.assert_allclose(d, cr.min(axis=1), rtol=1e-12, atol=1e-15)


def test_reference_permutation_permutes_pi():
    rng = np.random.default_rng(2)
    Z = wl.das_dennis(3, 8)
    perm = rng.permutation(len(Z))
    Fn = rng.random((500, 3))
    rank, fi = all_st(500)
    pi1, d1 = oracle.associate(Fn, rank, fi, Z)
    pi2, d2 = oracle.associate(Fn, rank, fi, Z[perm])
    inv = np.argsort(perm)
    # same reference chosen (ties are measure-zero for random points)
    assert np.array_equal(perm[pi2], pi1)
    np.testing.assert_array_equal(d1, d2)


def test_rows_outside_st():
    Z = wl.das_dennis(3, 4)
    Fn = np.ones((5, 3))
    rank = np.array([0, 1, 2, oracle.UNRANKED, 1], np.int32)
    fi = np.array([1, 1, 1, 3], np.int32)
    pi, d = oracle.associate(Fn, rank, fi, Z)
    assert list(pi[[2, 3]]) == [-1, -1]
    assert np.all(pi[[0, 1, 4]] >= 0)
