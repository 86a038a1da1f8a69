"""GPU parity of nsga3_normalize on pinned inputs (the oracle's ranks): ideal
point bit-exact (a float minimum), extreme points exact unless the FP64 ASF
gap is a near-tie, intercepts within FP64 rounding of the oracle when the
extremes agree (same elimination on the same matrix), Fn within FP32
rounding (relative 2e-6 of the row norm)."""
import numpy as np
import pytest

import oracle
from gpu_util import device, to_dev, to_np
from paper_2504_06067_amd import nsga3
from paper_2504_06067_amd import workloads as wl

pytestmark = pytest.mark.gpu


def asf64(F, z, x, k):
    fp = F[x].astype(np.float64) - z
    g = 1e6 * fp
    g[k] = fp[k]
    return g.max()


def compare(F, rank, fi, dev):
    ref = oracle.normalize(F, rank, fi)
    out = nsga3.normalize(to_dev(F, dev), to_dev(rank, dev), to_dev(fi, dev))
    ideal = to_np(out["ideal"])
    ext = to_np(out["extreme"])
    icpt = to_np(out["intercept"])
    deg = int(to_np(out["degenerate"])[0])
    Fn = to_np(out["Fn"])
    assert np.array_equal(ideal.astype(np.float64), ref["ideal"])
    z = ref["ideal"]
    near = 0
    for k in range(F.shape[1]):
        if ext[k] != ref["extreme"][k]:
            a, b = asf64(F, z, ext[k], k), asf64(F, z, ref["extreme"][k], k)
            assert abs(a - b) <= 1e-6 * max(abs(b), 1e-30), (k, a, b)
            near += 1
    if near == 0:
        assert deg == ref["degenerate"]
        np.testing.assert_allclose(icpt, ref["intercept"], rtol=1e-13)
        st = rank <= fi[0]
        scale = np.linalg.norm(ref["Fn"][st], axis=1, keepdims=True)
        err = np.abs(Fn[st].astype(np.float64) - ref["Fn"][st]) / np.maximum(scale, 1e-30)
        assert err.max() < 2e-6
    return near


@pytest.mark.parametrize("name,M,seed", [("small", None, 0), ("small", None, 1), ("large", 3000, 2),
                                         ("large", None, 0), ("many_objective", 5000, 0)])
def test_workloads(name, M, seed):
    dev = device()
    inst = wl.plain_instance(name, seed, M=M)
    rank, fi = oracle.nd_sort(inst["F"], inst["N"])
    assert compare(inst["F"], rank, fi, dev) == 0


@pytest.mark.parametrize("m", [2, 3, 5, 10, 16])
def test_random_objectives(m):
    dev = device()
    rng = np.random.default_rng(m)
    F = wl.objectives(rng, 3000, m, "exp")
    rank, fi = oracle.nd_sort(F, 1500)
    compare(F, rank, fi, dev)


def test_axis_identity():
    dev = device()
    rng = np.random.default_rng(3)
    m = 4
    F = np.concatenate([np.eye(m), 0.01 + rng.random((60, m))]).astype(np.float32)
    rank = np.zeros(len(F), np.int32)
    fi = np.array([0, 0, len(F), 1], np.int32)
    out = nsga3.normalize(to_dev(F, dev), to_dev(rank, dev), to_dev(fi, dev))
    assert np.array_equal(to_np(out["intercept"]), np.ones(m))
    assert np.array_equal(to_np(out["Fn"]), F)


def test_degenerate():
    dev = device()
    rng = np.random.default_rng(4)
    x = rng.random((80, 2))
    F = np.stack([x[:, 0], x[:, 1], x[:, 1]], axis=1).astype(np.float32)
    rank = np.zeros(80, np.int32)
    fi = np.array([0, 0, 80, 1], np.int32)
    out = nsga3.normalize(to_dev(F, dev), to_dev(rank, dev), to_dev(fi, dev))
    assert int(to_np(out["degenerate"])[0]) == 1
    ref = oracle.normalize(F, rank, fi)
    assert np.array_equal(to_np(out["intercept"]), ref["intercept"])


# The oracle's pinned degeneracy and tie cases (dyadic inputs, exact in
# float32): the GPU takes the same branch and gives the same intercepts.
def _run_all_st(F, dev):
    M = len(F)
    rank = np.zeros(M, np.int32)
    fi = np.array([0, 0, M, 1], np.int32)
    out = nsga3.normalize(to_dev(F, dev), to_dev(rank, dev), to_dev(fi, dev))
    ref = oracle.normalize(F, rank, fi)
    return ({k: to_np(v) for k, v in out.items()}, ref)


def test_asf_tie_least_index():
    dev = device()
    t = 2.0 ** -10
    base = [(1.0, 1.0, 1.0), (0.0, 1.0, 0.5), (0.75, 0.0, 1.0)]
    for lo, hi in ((0.5, 0.25), (0.25, 0.5)):
        F = np.array(base + [(lo, t, 0.0), (hi, t, 0.0)], np.float32)
        out, ref = _run_all_st(F, dev)
        assert int(out["extreme"][0]) == 3 == int(ref["extreme"][0])
        assert np.array_equal(out["extreme"], ref["extreme"])


@pytest.mark.parametrize("e3,extra,degen", [
    ((0.875, 0.875, 0.125), [], 1),            # b_3 = -6
    ((0.5, 0.5, 0.125), [], 1),                # b_3 = 0
    ((0.25, 0.25, 2.0 ** -20), [(2.0, 2.0, 4.0)], 1),  # a_3 = 2^-19 < 1e-6 * 4
    ((0.25, 0.25, 2.0 ** -20), [(2.0, 2.0, 1.0)], 0),  # a_3 = 2^-19 >= 1e-6 * 1
])
def test_degeneracy_branches(e3, extra, degen):
    dev = device()
    F = np.array([(1.0, 0.0, 0.0), (0.0, 1.0, 0.0), e3, *extra], np.float32)
    out, ref = _run_all_st(F, dev)
    assert ref["degenerate"] == degen
    assert int(out["degenerate"][0]) == degen
    assert np.array_equal(out["extreme"], ref["extreme"])
    assert np.array_equal(out["intercept"], ref["intercept"])
