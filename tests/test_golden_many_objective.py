"""The stored oracle selection of the many-objective workload is
self-consistent and agrees with the oracle's later stages and with
brute-force dominance (the sort that wrote it takes about a minute with 8
threads, so here it is checked on samples, plus the full later stages)."""
import hashlib
import os

import numpy as np

import oracle
from golden_data import many_objective_seed0
from paper_2504_06067_amd import workloads as wl


def dominators(F, x):
    le = np.all(F <= F[x], axis=1)
    lt = np.any(F < F[x], axis=1)
    return int(np.sum(le & lt))


def test_fixture_against_oracle_stages():
    fx = many_objective_seed0()
    inst = wl.plain_instance("many_objective", 0)
    F, Z, N = inst["F"], inst["Z"], inst["N"]
    assert fx["M"] == len(F) and fx["n_ranked"] == int(fx["ranked"].sum())
    assert len(fx["selected"]) == N and np.all(fx["ranked"][fx["selected"]])
    rng = np.random.default_rng(1)
    for x in rng.choice(np.where(fx["ranked"])[0], 40, replace=False):
        assert dominators(F, x) == 0
    for x in rng.choice(np.where(~fx["ranked"])[0], 40, replace=False):
        assert dominators(F, x) > 0
    rank = np.where(fx["ranked"], 0, oracle.UNRANKED).astype(np.int32)
    fi = fx["front_info"]
    try:
        oracle.set_threads(min(16, os.cpu_count() or 1))
        Fn = oracle.normalize(F, rank, fi)["Fn"]
        pi, d = oracle.associate(Fn, rank, fi, Z)
    finally:
        oracle.set_threads(1)
    assert hashlib.sha256(pi.astype("<i4").tobytes()).hexdigest() == fx["pi_sha256"]
    sel = oracle.niche(rank, fi, pi, d, len(Z), N, inst["seed"])
    assert np.array_equal(sel, fx["selected"])
