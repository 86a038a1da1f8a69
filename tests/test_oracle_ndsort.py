"""Pins for the oracle's non-dominated sort and front fill (paper Sec. II-C,
Algorithm 1 "Non-dominated-sort"): brute force on tiny inputs, rank
invariants, and closed forms."""
import numpy as np
import pytest

import oracle
from paper_2504_06067_amd import workloads as wl


def brute_ranks(F):
    """Naive peeling: repeatedly remove every point no remaining point dominates."""
    F = np.asarray(F, np.float64)
    M = len(F)
    alive = list(range(M))
    rank = [-1] * M
    k = 0
    while alive:
        front = []
        for j in alive:
            dominated = False
            for i in alive:
                if np.all(F[i] <= F[j]) and np.any(F[i] < F[j]):
                    dominated = True
                    break
            if not dominated:
                front.append(j)
        for j in front:
            rank[j] = k
        alive = [j for j in alive if j not in front]
        k += 1
    return np.array(rank)


@pytest.mark.parametrize("kind", ["continuous", "grid", "chain", "equal"])
@pytest.mark.parametrize("M,m", [(2, 2), (7, 2), (33, 3), (64, 4), (50, 6), (40, 32), (24, 512)])
def test_brute_force(kind, M, m):
    rng = np.random.default_rng(M * 100 + m)
    for trial in range(3):
        F = wl.random_small(rng, M, m, kind)
        rank, fi = oracle.nd_sort(F, 0)
        assert np.array_equal(rank, brute_ranks(F))
        assert fi[3] == rank.max() + 1


def dom_matrix(F):
    F = np.asarray(F, np.float64)
    le = np.all(F[:, None, :] <= F[None, :, :], axis=2)
    lt = np.any(F[:, None, :] < F[None, :, :], axis=2)
    return le & lt  # [i, j]: i dominates j


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_rank_invariants_small_workload(seed):
    inst = wl.plain_instance("small", seed)
    rank, fi = oracle.nd_sort(inst["F"], 0)
    D = dom_matrix(inst["F"])
    for r in range(rank.max() + 1):
        mem = np.where(rank == r)[0]
        assert not D[np.ix_(mem, mem)].any()          # same-rank points never dominate each other
        if r == 0:
            assert not D[:, mem].any()                # rank-0 points are non-dominated
        else:
            prev = np.where(rank == r - 1)[0]
            assert D[np.ix_(prev, mem)].any(axis=0).all()  # each has a dominator one rank up


def test_rank_invariants_many_fronts():
    inst = wl.plain_instance("large", 3, M=3000)
    rank, fi = oracle.nd_sort(inst["F"], 0)
    assert fi[3] > 5
    D = dom_matrix(inst["F"])
    for r in range(rank.max() + 1):
        mem = np.where(rank == r)[0]
        assert not D[np.ix_(mem, mem)].any()
        if r > 0:
            prev = np.where(rank == r - 1)[0]
            assert D[np.ix_(prev, mem)].any(axis=0).all()


def test_sphere_is_one_front():
    # equal norms: a <= b componentwise with a != b would force ||a|| < ||b||
    rng = np.random.default_rng(5)
    F = wl.directions(rng, 500, 5).astype(np.float32)
    F = F / np.linalg.norm(F.astype(np.float64), axis=1, keepdims=True)
    F = F.astype(np.float32)
    # float32 rounding can break exact equal norms; accept only if brute force agrees
    rank, fi = oracle.nd_sort(F, 0)
    D = dom_matrix(F)
    assert (rank == 0).sum() == (~D.any(axis=0)).sum()
    assert (rank == 0).sum() >= 490


def test_chain_gives_m_fronts():
    M = 40
    t = np.random.default_rng(1).permutation(M).astype(np.float32)
    F = np.repeat(t[:, None], 3, axis=1)
    rank, fi = oracle.nd_sort(F, 0)
    assert np.array_equal(rank, t.astype(int))
    assert fi[3] == M


@pytest.mark.parametrize("n_stop", [1, 5, 17, 40, 63, 64])
def test_front_fill(n_stop):
    rng = np.random.default_rng(n_stop)
    F = wl.random_small(rng, 64, 3, "grid")
    full, _ = oracle.nd_sort(F, 0)
    rank, fi = oracle.nd_sort(F, n_stop)
    sizes = np.bincount(full)
    cum = np.cumsum(sizes)
    l = int(np.argmax(cum >= n_stop))
    S = int(cum[l - 1]) if l > 0 else 0
    assert list(fi[:3]) == [l, S, n_stop - S]
    assert 1 <= fi[2] <= sizes[l]
    assert np.array_equal(rank[full <= l], full[full <= l])
    assert np.all(rank[full > l] == oracle.UNRANKED)


def test_large_workload_front_structure():
    # regression anchor of the exponential-radius law at 2N = 20000 (seed 0):
    # nine fronts reach N = 10000
    inst = wl.plain_instance("large", 0)
    rank, fi = oracle.nd_sort(inst["F"], inst["N"])
    assert list(fi[:3]) == [8, 9306, 694]
    assert (rank == 8).sum() == 946


def test_rejects_nonfinite():
    F = np.ones((4, 2), np.float32)
    F[2, 1] = np.nan
    with pytest.raises(RuntimeError):
        oracle.nd_sort(F, 0)


@pytest.mark.parametrize("name,M,seed", [("small", None, 0), ("large", 3000, 1),
                                         ("many_objective", 2500, 2)])
def test_threads_do_not_change_results(name, M, seed):
    # the multi-threaded dominance (ordered pairs, row by row) and association
    # loops give the serial oracle's results exactly
    inst = wl.plain_instance(name, seed, M=M)
    F = inst["F"].copy()
    F[7] = F[3]  # a duplicate pair: mutually non-dominating
    try:
        oracle.set_threads(1)
        a = oracle.select(F, inst["Z"], inst["N"], inst["seed"])
        oracle.set_threads(4)
        b = oracle.select(F, inst["Z"], inst["N"], inst["seed"])
    finally:
        oracle.set_threads(1)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
