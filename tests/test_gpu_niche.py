"""GPU parity of nsga3_niche (and of the cache-tensor baseline,
nsga3_niche_cache_tensor) on pinned inputs: identical (rank, front_info,
pi, dist) go to the GPU and to the oracle's sequential loop; the selected
sets must be identical (integer result)."""
import numpy as np
import pytest

import oracle
from gpu_util import device, to_dev, to_np
from paper_2504_06067_amd import nsga3

pytestmark = pytest.mark.gpu


def make_case(rng, M, H, nfront, dist_ties=True):
    sizes = np.maximum(rng.multinomial(M, np.ones(nfront) / nfront), 1)
    M = int(sizes.sum())
    rank = np.repeat(np.arange(nfront), sizes).astype(np.int32)
    rng.shuffle(rank)
    N = int(rng.integers(1, M + 1))
    cum = np.cumsum(sizes)
    l = int(np.argmax(cum >= N))
    S = int(cum[l - 1]) if l > 0 else 0
    rank = np.where(rank > l, oracle.UNRANKED, rank).astype(np.int32)
    fi = np.array([l, S, N - S, l + 1], np.int32)
    pi = rng.integers(0, H, M).astype(np.int32)
    pi[rank > l] = -1
    dist = rng.random(M).astype(np.float32)
    if dist_ties:
        dist[rng.random(M) < 0.3] = np.float32(0.25)
    return rank, fi, pi, dist, N


def check(rank, fi, pi, dist, H, N, seed, dev):
    """The closed form (nsga3_niche) and the paper's cache-tensor loop
    (nsga3_niche_cache_tensor) both equal the oracle's sequential loop."""
    ref = oracle.niche(rank, fi, pi, dist.astype(np.float64), H, N, seed)
    args = (to_dev(rank, dev), to_dev(fi, dev), to_dev(pi, dev), to_dev(dist, dev), H, N, seed)
    sel = to_np(nsga3.niche(*args))
    assert np.array_equal(sel, ref)
    ct = to_np(nsga3.niche(*args, cache_tensor=True))
    assert np.array_equal(ct, ref), "cache-tensor loop differs from the oracle"


@pytest.mark.parametrize("case", range(60))
def test_random_cases(case):
    dev = device()
    rng = np.random.default_rng(case)
    M = int(rng.integers(2, 3000))
    H = int(rng.integers(1, 300))
    rank, fi, pi, dist, N = make_case(rng, M, H, int(rng.integers(1, 6)))
    check(rank, fi, pi, dist, H, N, case * 1315423911, dev)


@pytest.mark.parametrize("H", [1, 2, 3])
def test_few_references_long_segments(H):
    # segments longer than the per-wave LDS capacity take the global-memory path
    dev = device()
    rng = np.random.default_rng(H)
    M = 12000
    rank = np.zeros(M, np.int32)
    rank[rng.random(M) < 0.6] = 1
    fi = np.array([1, int((rank == 0).sum()), 0, 2], np.int32)
    N = int(fi[1] + 0.6 * (rank == 1).sum()) if H > 1 else int(fi[1] + 300)
    fi[2] = N - fi[1]
    pi = rng.integers(0, H, M).astype(np.int32)
    dist = rng.random(M).astype(np.float32)
    check(rank, fi, pi, dist, H, N, 99 + H, dev)


def test_single_front_all_level_zero():
    # S is empty: every reference starts at niche count 0 (nearest picks), then random
    dev = device()
    rng = np.random.default_rng(7)
    M, H = 5000, 400
    rank = np.zeros(M, np.int32)
    fi = np.array([0, 0, 2500, 1], np.int32)
    pi = rng.integers(0, H, M).astype(np.int32)
    dist = rng.random(M).astype(np.float32)
    check(rank, fi, pi, dist, H, 2500, 3, dev)


def test_whole_last_front_taken():
    dev = device()
    rng = np.random.default_rng(8)
    M, H = 1000, 50
    rank = np.where(rng.random(M) < 0.5, 0, 1).astype(np.int32)
    nS = int((rank == 0).sum())
    nF = int((rank == 1).sum())
    fi = np.array([1, nS, nF, 2], np.int32)
    pi = rng.integers(0, H, M).astype(np.int32)
    dist = rng.random(M).astype(np.float32)
    check(rank, fi, pi, dist, H, nS + nF, 4, dev)


def test_many_levels():
    # crowded S so that L* is high and several levels are filled
    dev = device()
    rng = np.random.default_rng(9)
    M, H = 20000, 64
    rank = np.where(rng.random(M) < 0.7, 0, 1).astype(np.int32)
    nS = int((rank == 0).sum())
    nF = int((rank == 1).sum())
    K = nF // 2
    fi = np.array([1, nS, K, 2], np.int32)
    pi = rng.integers(0, H, M).astype(np.int32)
    pi[(rank == 0) & (pi < 8)] = 9  # refs 0..7 have no S members: level-0 picks
    dist = rng.random(M).astype(np.float32)
    check(rank, fi, pi, dist, H, nS + K, 5, dev)


@pytest.mark.parametrize("H", [1025, 12288, 12289, 30000])
def test_reference_rows_and_groups(H):
    # several rows of plan threads, and more references than one group of rows
    dev = device()
    rng = np.random.default_rng(H)
    M = 3 * H
    rank = np.where(rng.random(M) < 0.5, 0, 1).astype(np.int32)
    nS = int((rank == 0).sum())
    nF = int((rank == 1).sum())
    K = nF // 3
    fi = np.array([1, nS, K, 2], np.int32)
    pi = rng.integers(0, H, M).astype(np.int32)
    dist = rng.random(M).astype(np.float32)
    check(rank, fi, pi, dist, H, nS + K, 11 + H, dev)
