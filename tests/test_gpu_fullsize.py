"""Full-size workloads in the launch configuration that bench.py times.

The many-objective workload (2N = 131072, m = 10, H = 2002, N = 65536) is out
of reach for the oracle's O(M^2 m) sort, so its ranks are checked on samples
against brute-force dominance over all points (a rank-0 point has no
dominator; an unranked point has one, since front 0 alone fills N here), and
the later stages by pinned-stage parity: the oracle's FP64 normalization and
association run on the GPU's ranks, and the oracle's niching on the GPU's
(rank, pi, dist) must give the GPU's selection exactly. The large workload at
full size is compared with the oracle end to end in test_gpu_select."""
import numpy as np
import pytest

import oracle
from gpu_util import association_report, device, to_dev, to_np
from paper_2504_06067_amd import nsga3
from paper_2504_06067_amd import workloads as wl

pytestmark = pytest.mark.gpu


def dominators(F, x):
    """Number of points that dominate point x (brute force, float compares)."""
    le = np.all(F <= F[x], axis=1)
    lt = np.any(F < F[x], axis=1)
    return int(np.sum(le & lt))


def test_many_objective_full_size():
    dev = device()
    inst = wl.plain_instance("many_objective", 0)
    F, Z, N, M = inst["F"], inst["Z"], inst["N"], inst["M"]
    out = nsga3.select(to_dev(F, dev), to_dev(Z, dev), N, inst["seed"], intermediates=True)
    g = {k: to_np(v) for k, v in out.items()}
    rank = g["rank"]
    ranked = rank != nsga3.UNRANKED
    # front 0 alone holds at least N points at this workload: l = 0, S empty
    assert np.all(rank[ranked] == 0)
    n0 = int(ranked.sum())
    assert n0 >= N
    fi = np.array([0, 0, N, 1], dtype=np.int32)
    rng = np.random.default_rng(0)
    for x in rng.choice(np.where(ranked)[0], 200, replace=False):
        assert dominators(F, x) == 0, x
    for x in rng.choice(np.where(~ranked)[0], 200, replace=False):
        assert dominators(F, x) > 0, x
    # normalization and association: the oracle on the GPU's ranks
    Fn = oracle.normalize(F, rank, fi)["Fn"]
    pi_ref, d_ref = oracle.associate(Fn, rank, fi, Z)
    st = np.where(ranked)[0]
    nmis, nflag, derr = association_report(np.nan_to_num(Fn, nan=0.0), Z, st, g["pi"], pi_ref,
                                           g["dist"], d_ref)
    assert nmis == nflag, f"{nmis - nflag} association mismatches outside the near-tie band"
    assert nflag <= max(2, 1e-3 * len(st))
    assert derr < 1e-6
    # niching on the GPU's own intermediates
    chained = oracle.niche(rank, fi, g["pi"], g["dist"].astype(np.float64), len(Z), N,
                           inst["seed"])
    assert np.array_equal(g["selected"], chained)


def test_large_full_size_front_counts():
    """The large workload's front structure at full size (nine selected
    fronts; the front fill of the paper's selection)."""
    dev = device()
    inst = wl.plain_instance("large", 0)
    rank, fi = nsga3.nd_sort(to_dev(inst["F"], dev), inst["N"])
    rank, fi = to_np(rank), to_np(fi)
    l = int(fi[0])
    sizes = [int(np.sum(rank == k)) for k in range(l + 1)]
    assert fi[1] == sum(sizes[:l]) and fi[2] == inst["N"] - fi[1] and fi[3] == l + 1
    assert sum(sizes[:l]) < inst["N"] <= sum(sizes)
    ref_rank, ref_fi = oracle.nd_sort(inst["F"], inst["N"])
    assert np.array_equal(fi, ref_fi) and np.array_equal(rank, ref_rank)
