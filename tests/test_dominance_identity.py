"""The compare identities the dominance kernel's tiles use, checked by brute
force on the CPU (the kernels are checked end to end by the GPU parity
tests).

For points i and j (minimization, float32 compares, no NaN):
  * full tiles: "i dominates j" is (some objective less) and not (some
    objective greater); from five objectives the kernel forms it as
    (every objective <=) and not (every objective >=), and "j dominates i"
    as (every >=) and not (every <=);
  * ordered tiles (f_1(i) < f_1(j) by the placement): "i dominates j" is
    every objective 2 .. m <=.
"""
import numpy as np
import pytest


def dominates(a, b):
    return bool(np.all(a <= b) and np.any(a < b))


def cases(m, seed):
    rng = np.random.default_rng(seed)
    grid = rng.integers(0, 3, (300, m)).astype(np.float32)
    z = grid.copy()
    z[(z == 0) & (rng.random(z.shape) < 0.5)] = np.float32(-0.0)
    inf = rng.random((300, m)).astype(np.float32)
    inf[rng.random(inf.shape) < 0.1] = np.float32(np.inf)
    inf[rng.random(inf.shape) < 0.1] = np.float32(-np.inf)
    return [rng.random((300, m)).astype(np.float32), grid, z, inf]


@pytest.mark.parametrize("m", [2, 3, 5, 8, 16])
def test_full_tile_identity(m):
    for F in cases(m, m):
        for i in range(0, 300, 7):
            a = F[i]
            lt = np.any(a < F, axis=1)
            gt = np.any(a > F, axis=1)
            le = np.all(a <= F, axis=1)
            ge = np.all(a >= F, axis=1)
            assert np.array_equal(lt & ~gt, le & ~ge)
            assert np.array_equal(gt & ~lt, ge & ~le)
            ref_ij = np.array([dominates(a, b) for b in F])
            ref_ji = np.array([dominates(b, a) for b in F])
            assert np.array_equal(le & ~ge, ref_ij)
            assert np.array_equal(ge & ~le, ref_ji)


@pytest.mark.parametrize("m", [2, 3, 5, 8, 16])
def test_ordered_tile_identity(m):
    for F in cases(m, 100 + m):
        for i in range(0, 300, 7):
            a = F[i]
            first_less = a[0] < F[:, 0]
            rest_le = np.all(a[1:] <= F[:, 1:], axis=1)
            ref = np.array([dominates(a, b) for b in F])
            # where the placement guarantees f_1(i) < f_1(j), the check of
            # objectives 2 .. m alone decides
            assert np.array_equal(rest_le[first_less], ref[first_less])
