"""GPU parity of nsga3_nd_sort against the oracle: ranks and front_info
bit-exact (integer results), across tile boundaries, ragged tails, ties,
duplicates, chains, early stops and the full-size workloads."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import device, to_dev, to_np
from paper_2504_06067_amd import nsga3
from paper_2504_06067_amd import workloads as wl

pytestmark = pytest.mark.gpu


def run(F, n_stop, dev, ws=None):
    rank, fi = nsga3.nd_sort(to_dev(F, dev), n_stop, ws=ws)
    return to_np(rank), to_np(fi)


@pytest.mark.parametrize("kind", ["continuous", "grid", "chain", "equal"])
@pytest.mark.parametrize("M,m", [(2, 2), (3, 3), (63, 2), (64, 3), (65, 4), (127, 5), (129, 8),
                                 (200, 16), (640, 3), (1000, 10)])
def test_ranks_exact(kind, M, m):
    dev = device()
    rng = np.random.default_rng(M * 31 + m)
    F = wl.random_small(rng, M, m, kind)
    ref_rank, ref_fi = oracle.nd_sort(F, 0)
    rank, fi = run(F, 0, dev)
    assert np.array_equal(rank, ref_rank)
    assert np.array_equal(fi, ref_fi)


@pytest.mark.parametrize("kind", ["continuous", "grid", "signed_zero"])
@pytest.mark.parametrize("m", list(range(5, 17)))
def test_ordered_tiles_every_m(kind, m):
    """Every compare count of the ordered tiles' EXEC-chained compares (m - 1
    of them, m = 5 .. 16): 777 points (13 blocks, a ragged last one), most
    tiles ordered by the first-objective placement; ties on a grid, and
    -0.0 against +0.0 in every objective."""
    dev = device()
    rng = np.random.default_rng(1000 + m)
    if kind == "continuous":
        F = rng.random((777, m)).astype(np.float32)
    else:
        F = rng.integers(0, 4, (777, m)).astype(np.float32)
        if kind == "signed_zero":
            F[(F == 0) & (rng.random(F.shape) < 0.5)] = np.float32(-0.0)
    ref_rank, ref_fi = oracle.nd_sort(F, 0)
    rank, fi = run(F, 0, dev)
    assert np.array_equal(rank, ref_rank)
    assert np.array_equal(fi, ref_fi)


@pytest.mark.parametrize("n_stop", [1, 7, 100, 500, 999, 1000])
def test_early_stop(n_stop):
    dev = device()
    inst = wl.plain_instance("large", 11, M=1000)
    ref_rank, ref_fi = oracle.nd_sort(inst["F"], n_stop)
    rank, fi = run(inst["F"], n_stop, dev)
    assert np.array_equal(fi, ref_fi)
    assert np.array_equal(rank, ref_rank)


@pytest.mark.parametrize("name,M", [("small", None), ("large", 4000), ("large", None),
                                    ("many_objective", 6000)])
def test_workloads(name, M):
    dev = device()
    for seed in ([0, 1, 2] if name == "small" else [0]):
        inst = wl.plain_instance(name, seed, M=M)
        ref_rank, ref_fi = oracle.nd_sort(inst["F"], inst["N"])
        rank, fi = run(inst["F"], inst["N"], dev)
        assert np.array_equal(fi, ref_fi), (fi, ref_fi)
        assert np.array_equal(rank, ref_rank)


def test_workspace_reuse_is_deterministic():
    dev = device()
    ws = nsga3.Workspace(dev)
    inst = wl.plain_instance("large", 5, M=3000)
    a = run(inst["F"], inst["N"], dev, ws)
    b = run(inst["F"], inst["N"], dev, ws)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_nonfinite_sets_status():
    dev = device()
    F = np.random.default_rng(0).random((100, 3)).astype(np.float32)
    F[17, 2] = np.nan
    ws = nsga3.Workspace(dev)
    nsga3.nd_sort(to_dev(F, dev), 50, ws=ws)
    torch.cuda.synchronize()
    assert ws.status() == nsga3.ENONFINITE
    F[17, 2] = 0.5
    nsga3.nd_sort(to_dev(F, dev), 50, ws=ws)
    assert ws.status() == nsga3.OK


# Sizes that select each way the peel holds a chunk's matrix column: in
# registers, 16 .. 48 words per wave (W = ceil(M / 64) up to 8 x 16 .. 8 x 48,
# at most two chunks per compute unit), or streamed from memory every front
# (W above 384). Each instance has many fronts (radius law "exp").
@pytest.mark.parametrize("M", [6000, 9000, 15000, 20000, 24500, 25600])
def test_peel_column_paths(M):
    dev = device()
    rng = np.random.default_rng(M)
    F = wl.objectives(rng, M, 3, "exp")
    ref_rank, ref_fi = oracle.nd_sort(F, 0)
    rank, fi = run(F, 0, dev)
    assert ref_fi[3] > 5  # several fronts
    assert np.array_equal(rank, ref_rank)
    assert np.array_equal(fi, ref_fi)
