"""Full-size workloads in the launch configuration that bench.py times.

The many-objective workload (2N = 131072, m = 10, H = 2002, N = 65536):
the oracle's sort at this size takes about a minute on 8 cores, so its full
selection was stored once (tests/golden/many_objective_seed0.txt, written by
an oracle-only script); the GPU's ranks and selection are compared with it
element by element, and the later stages with the oracle run here on the
GPU's ranks. The large workload at full size is compared with the oracle end
to end in test_gpu_select."""
import hashlib
import os

import numpy as np
import pytest

import oracle
from golden_data import many_objective_seed0
from gpu_util import association_report, device, to_dev, to_np
from paper_2504_06067_amd import nsga3
from paper_2504_06067_amd import workloads as wl

pytestmark = pytest.mark.gpu


def test_many_objective_full_size():
    """Ranks and selection against the stored FP64 oracle selection
    (tests/golden/many_objective_seed0.txt), element by element."""
    dev = device()
    fx = many_objective_seed0()
    inst = wl.plain_instance("many_objective", 0)
    F, Z, N, M = inst["F"], inst["Z"], inst["N"], inst["M"]
    out = nsga3.select(to_dev(F, dev), to_dev(Z, dev), N, inst["seed"], intermediates=True)
    g = {k: to_np(v) for k, v in out.items()}
    rank = g["rank"]
    ranked = rank != nsga3.UNRANKED
    # ranks: every point, bit-exact (one ranked front at this workload)
    assert np.array_equal(ranked, fx["ranked"])
    assert np.all(rank[ranked] == 0)
    fi = fx["front_info"]
    # the oracle's FP64 normalization and association at these ranks
    try:
        oracle.set_threads(min(16, os.cpu_count() or 1))
        nrm = oracle.normalize(F, rank, fi)
        pi_ref, d_ref = oracle.associate(nrm["Fn"], rank, fi, Z)
    finally:
        oracle.set_threads(1)
    assert hashlib.sha256(pi_ref.astype("<i4").tobytes()).hexdigest() == fx["pi_sha256"]
    ext = to_np(nsga3.normalize(to_dev(F, dev), to_dev(rank, dev), to_dev(fi, dev))["extreme"])
    assert np.array_equal(ext, nrm["extreme"])
    st = np.where(ranked)[0]
    nmis, nflag, derr = association_report(np.nan_to_num(nrm["Fn"], nan=0.0), Z, st, g["pi"],
                                           pi_ref, g["dist"], d_ref)
    assert nmis == nflag, f"{nmis - nflag} association mismatches outside the near-tie band"
    assert nflag <= max(2, 1e-3 * len(st))
    assert derr < 1e-6
    # niching on the GPU's own intermediates, and the stored selection when
    # no association was flagged
    chained = oracle.niche(rank, fi, g["pi"], g["dist"].astype(np.float64), len(Z), N,
                           inst["seed"])
    assert np.array_equal(g["selected"], chained)
    if nflag == 0:
        assert np.array_equal(g["selected"], fx["selected"])
    print(f"many-objective full size: {nflag} flagged association near-ties of {len(st)}, "
          f"max distance error {derr:.2e} of ||f_n||", flush=True)


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
