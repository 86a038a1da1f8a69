"""The one-workgroup selection of small instances (nsga3_select below the
tiny work budget) against the multi-kernel path (the same instance through
nsga3_select_batched, which always runs the multi-kernel path): rank, pi,
dist and the selection bit for bit, plus the FP64 oracle's bar; error
statuses; and the shapes at the edge of the budget."""
import numpy as np
import pytest
import torch

from gpu_util import device, select_parity, to_dev, to_np
from paper_2504_06067_amd import nsga3
from paper_2504_06067_amd import workloads as wl

pytestmark = pytest.mark.gpu

KEYS = ("selected", "rank", "pi", "dist")


def both(F, Z, N, seed, dev):
    Fd, Zd = to_dev(F, dev), to_dev(Z, dev)
    tiny = nsga3.select(Fd, Zd, N, seed, intermediates=True)
    bt = nsga3.Batch([dict(F=Fd, Z=Zd, N=N, seed=seed)], intermediates=True)
    bt.run()
    torch.cuda.synchronize(dev)
    assert bt.status() == [nsga3.OK]
    big = {k: getattr(bt, k)[0] for k in KEYS}
    return {k: to_np(v) for k, v in tiny.items()}, {k: to_np(v) for k, v in big.items()}


def check(F, Z, N, seed, dev, oracle_bar=True):
    print(f"tiny: M={len(F)} m={F.shape[1]} H={len(Z)} N={N}", flush=True)
    t, b = both(F, Z, N, seed, dev)
    for k in KEYS:
        assert np.array_equal(t[k], b[k]), k
    if oracle_bar:
        select_parity(dict(F=F, Z=Z, N=N, seed=seed), t, dev)


@pytest.mark.parametrize("M,m,p", [(2, 2, 1), (3, 2, 3), (64, 3, 12), (65, 3, 12), (130, 5, 4),
                                   (184, 3, 12), (200, 6, 4), (256, 3, 12), (255, 4, 6),
                                   (120, 10, 2), (90, 16, 1), (256, 2, 60)])
def test_tiny_equals_multi_kernel(M, m, p):
    dev = device()
    F = wl.objectives(np.random.default_rng(M * 31 + m), M, m, "exp")
    Z = wl.das_dennis(m, p)
    for N in sorted({1, max(1, M // 2), M}):
        check(F, Z, N, N + m, dev)


@pytest.mark.parametrize("seed", range(6))
def test_small_workload_seeds(seed):
    dev = device()
    inst = wl.plain_instance("small", seed)
    check(inst["F"], inst["Z"], inst["N"], seed, dev)


def test_ties_chains_and_duplicates():
    dev = device()
    rng = np.random.default_rng(5)
    # a chain: every point dominates the next, one point per front
    M = 200
    F = np.repeat(np.arange(M, dtype=np.float32)[:, None], 3, axis=1)
    Z = wl.das_dennis(3, 6)
    check(F, Z, 150, 1, dev)
    # exact duplicates and a coarse grid (many ties in every objective)
    F = rng.integers(0, 4, (240, 3)).astype(np.float32)
    check(F, Z, 120, 2, dev, oracle_bar=False)
    # all points equal: one front, degenerate normalization
    F = np.ones((100, 4), np.float32)
    check(F, wl.das_dennis(4, 3), 37, 3, dev, oracle_bar=False)
    # one reference
    F = wl.objectives(rng, 150, 3, "exp")
    check(F, np.ones((1, 3), np.float32), 70, 4, dev)


def test_error_statuses():
    dev = device()
    inst = wl.plain_instance("small", 0)
    ws = nsga3.Workspace(dev)
    F = inst["F"].copy()
    F[5, 2] = np.inf
    nsga3.select(to_dev(F, dev), to_dev(inst["Z"], dev), inst["N"], 0, ws=ws)
    assert ws.status() == nsga3.ENONFINITE
    Z = inst["Z"].copy()
    Z[3] = 0.0
    nsga3.select(to_dev(inst["F"], dev), to_dev(Z, dev), inst["N"], 0, ws=ws)
    assert ws.status() == nsga3.EINVAL
    nsga3.select(to_dev(inst["F"], dev), to_dev(inst["Z"], dev), inst["N"], 0, ws=ws)
    assert ws.status() == nsga3.OK


def test_edge_of_the_budget():
    # just inside and just outside the one-workgroup limits give the same results
    dev = device()
    for M, m, p in [(256, 4, 6), (257, 4, 6), (300, 3, 12)]:
        F = wl.objectives(np.random.default_rng(M), M, m, "exp")
        check(F, wl.das_dennis(m, p), M // 2, 7, dev)
