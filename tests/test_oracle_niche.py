"""Pins for the oracle's niching (Algorithm 1 loop; Algorithm 2 nearest and
random selection): an independent closed-form model, invariants, exhaustive
enumeration of the paper's random choices, and a chi-square test."""
import numpy as np
import pytest

import oracle
from niche_model import enumerate_outcomes, key, waterfill
from paper_2504_06067_amd import workloads as wl


def random_case(rng, M, H, nfront=3):
    """Synthetic (rank, front_info, pi, dist) with a partially selected last front."""
    sizes = rng.multinomial(M, np.ones(nfront) / nfront)
    sizes = np.maximum(sizes, 1)
    M = int(sizes.sum())
    rank = np.repeat(np.arange(nfront), sizes).astype(np.int32)
    rng.shuffle(rank)
    N = int(rng.integers(1, M + 1))
    cum = np.cumsum(sizes)
    l = int(np.argmax(cum >= N))
    S = int(cum[l - 1]) if l > 0 else 0
    rank = np.where(rank > l, oracle.UNRANKED, rank).astype(np.int32)
    fi = np.array([l, S, N - S, nfront], np.int32)
    pi = rng.integers(0, H, M).astype(np.int32)
    dist = rng.random(M)
    dist[rng.random(M) < 0.2] = 0.5          # exact distance ties
    return rank, fi, pi, dist, N


def test_key_model_matches_oracle_key():
    for s in [0, 1, 2**63 + 5]:
        for j in [0, 1, 77, 2**32 - 1]:
            for L in [0, 1, 2**30 - 1]:
                for tag in [1, 2]:
                    assert key(s, tag, j, L) == oracle.key(s, tag, j, L)


@pytest.mark.parametrize("seed", range(40))
def test_sequential_equals_waterfill(seed):
    rng = np.random.default_rng(seed)
    M = int(rng.integers(2, 300))
    H = int(rng.integers(1, 40))
    rank, fi, pi, dist, N = random_case(rng, M, H, int(rng.integers(1, 5)))
    sel = oracle.niche(rank, fi, pi, dist, H, N, seed * 7919)
    assert np.array_equal(sel, waterfill(rank, fi, pi, dist, H, seed * 7919))


@pytest.mark.parametrize("seed", range(10))
def test_invariants(seed):
    rng = np.random.default_rng(100 + seed)
    rank, fi, pi, dist, N = random_case(rng, 400, 30)
    sel = oracle.niche(rank, fi, pi, dist, 30, N, seed)
    l = fi[0]
    assert len(sel) == N and np.all(np.diff(sel) > 0)
    S = set(np.where(rank < l)[0])
    Fl = set(np.where(rank == l)[0])
    assert S <= set(sel) <= S | Fl
    picks = sorted(set(sel) - S)
    cnt = np.bincount(pi[sorted(S)], minlength=30) if S else np.zeros(30, int)
    final = cnt + np.bincount(pi[picks], minlength=30)
    cap = np.bincount(pi[sorted(Fl)], minlength=30)
    left = cap - np.bincount(pi[picks], minlength=30)
    # balance: a reference that kept candidates is never below a reference that got picks
    if len(picks):
        top = max(final[j] for j in set(pi[picks]))
        for j in range(30):
            if left[j] > 0:
                assert final[j] >= top - 1
    # level-0 picks are the nearest candidate of their reference
    for j in set(pi[picks]):
        if cnt[j] == 0:
            cand = [x for x in Fl if pi[x] == j]
            nearest = min(cand, key=lambda x: (dist[x], x))
            assert nearest in sel


def tiny_case(rng):
    M = int(rng.integers(4, 9))
    H = int(rng.integers(1, 4))
    rank = np.zeros(M, np.int32)
    nS = int(rng.integers(0, M - 2))
    rank[rng.permutation(M)[:nS]] = -1  # placeholder for S
    l = 1 if nS else 0
    rank = np.where(rank == -1, 0, l).astype(np.int32) if nS else rank
    Fl = int((rank == l).sum())
    K = int(rng.integers(1, Fl + 1))
    N = nS + K
    fi = np.array([l, nS, K, l + 1], np.int32)
    pi = rng.integers(0, H, M).astype(np.int32)
    dist = rng.random(M)
    return rank, fi, pi, dist, H, N


@pytest.mark.parametrize("case", range(25))
def test_oracle_result_is_a_possible_nsga3_outcome(case):
    rng = np.random.default_rng(1000 + case)
    rank, fi, pi, dist, H, N = tiny_case(rng)
    support = enumerate_outcomes(rank, fi, pi, dist, H)
    assert abs(sum(support.values()) - 1) == 0
    for s in range(30):
        sel = oracle.niche(rank, fi, pi, dist, H, N, s)
        assert tuple(sel) in support


def test_chi_square_against_exact_distribution():
    # a case with several random choices: two references, one already crowded
    rank = np.array([0, 0, 1, 1, 1, 1, 1, 1], np.int32)
    pi = np.array([0, 1, 0, 0, 1, 1, 1, 2], np.int32)
    dist = np.arange(8, dtype=np.float64)
    fi = np.array([1, 2, 3, 2], np.int32)
    H, N = 3, 5
    support = enumerate_outcomes(rank, fi, pi, dist, H)
    assert len(support) >= 4
    n = 20000
    counts = {}
    for s in range(n):
        t = tuple(oracle.niche(rank, fi, pi, dist, H, N, s))
        counts[t] = counts.get(t, 0) + 1
    assert set(counts) <= set(support)
    chi2 = sum((counts.get(t, 0) - n * float(p)) ** 2 / (n * float(p)) for t, p in support.items())
    dof = len(support) - 1
    # 0.1% upper quantile of chi-square, Wilson-Hilferty approximation
    z = 3.09
    crit = dof * (1 - 2 / (9 * dof) + z * (2 / (9 * dof)) ** 0.5) ** 3
    assert chi2 < crit, (chi2, crit, dof)


def test_select_small_workload():
    inst = wl.plain_instance("small", 0)
    r = oracle.select(inst["F"], inst["Z"], inst["N"], 0)
    rank, fi = oracle.nd_sort(inst["F"], inst["N"])
    assert np.array_equal(r["rank"], rank)
    sel = r["selected"]
    assert len(sel) == inst["N"] and np.all(np.diff(sel) > 0)
    assert set(np.where(rank < fi[0])[0]) <= set(sel)
    assert np.all(rank[sel] <= fi[0])
