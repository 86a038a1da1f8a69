"""Device quality indicators against the reference ones (oracle/quality_ref.py):
IGD within 1e-6 relative (FP32 distances, FP64 mean), the hypervolume sample
count exactly (identical FP32 sample points and decisions)."""
import numpy as np
import pytest
import torch

from gpu_util import device, to_dev, to_np
from oracle import quality_ref as q
from paper_2504_06067_amd import nsga3
from paper_2504_06067_amd import workloads as wl

pytestmark = pytest.mark.gpu


def unit(Z):
    Z = Z.astype(np.float64)
    return (Z / np.linalg.norm(Z, axis=1, keepdims=True)).astype(np.float32)


@pytest.mark.parametrize("n,m,p", [(1, 3, 12), (7, 2, 5), (1000, 3, 12), (4097, 5, 8),
                                   (3000, 10, 3), (50000, 3, 40), (600, 16, 1)])
def test_igd_matches_reference(n, m, p):
    dev = device()
    print(f"igd n={n} m={m}", flush=True)
    F = wl.objectives(np.random.default_rng(n + m), n, m, "exp")
    R = unit(wl.das_dennis(m, p))
    got = float(to_np(nsga3.igd(to_dev(F, dev), to_dev(R, dev)))[0])
    want = q.igd(F, R)
    assert abs(got - want) <= 1e-6 * (1.0 + want), (got, want)


def test_igd_of_the_front_is_zero():
    dev = device()
    R = unit(wl.das_dennis(3, 12))
    assert float(to_np(nsga3.igd(to_dev(R, dev), to_dev(R, dev)))[0]) == 0.0


@pytest.mark.parametrize("n,m,samples", [(1, 3, 1000), (5, 2, 4097), (300, 3, 20000),
                                         (2000, 5, 20000), (700, 10, 10000), (150, 15, 6000),
                                         (400, 16, 3001)])
def test_hv_count_matches_reference(n, m, samples):
    dev = device()
    print(f"hv n={n} m={m} samples={samples}", flush=True)
    F = wl.objectives(np.random.default_rng(10 * n + m), n, m, "exp")
    ideal, ref = q.hv_box(F.min(axis=0), F.max(axis=0))
    ref = ref.copy()
    # some points lie outside the box (n = 1: a box of zero width in objective 0)
    ref[0] = max(ideal[0], np.float32(0.8) * ref[0])
    got = int(to_np(nsga3.hv_count(to_dev(F, dev), ideal, ref, samples, seed=n))[0])
    assert got == q.hv_count(F, ideal, ref, samples, n)


def test_hv_rejects_an_inverted_box():
    dev = device()
    F = torch.ones((4, 3), dtype=torch.float32, device=dev)
    with pytest.raises(nsga3.Nsga3Error):
        nsga3.hv_count(F, [1, 0, 0], [0, 1, 1], 100, 0)
