"""nsga3_select_noalloc (the library's own per-GPU scratch, no workspace
argument) gives exactly what nsga3_select gives with a caller workspace, on
two calls in a row, the second on a smaller input (the scratch keeps the
first call's contents), and rejects shapes beyond the scratch."""
import numpy as np
import pytest
import torch

from gpu_util import device, to_dev, to_np
from paper_2504_06067_amd import nsga3
from paper_2504_06067_amd import workloads as wl

pytestmark = pytest.mark.gpu

KEYS = ("selected", "rank", "pi", "dist")


def _both(inst, dev):
    F, Z = to_dev(inst["F"], dev), to_dev(inst["Z"], dev)
    print(f"noalloc: M={inst['M']} m={inst['m']} H={inst['H']} N={inst['N']}", flush=True)
    ref = nsga3.select(F, Z, inst["N"], inst["seed"], intermediates=True)
    got, st = nsga3.select_noalloc(F, Z, inst["N"], inst["seed"], intermediates=True)
    torch.cuda.synchronize(dev)
    return {k: to_np(v) for k, v in ref.items()}, {k: to_np(v) for k, v in got.items()}, \
        int(to_np(st)[0])


def test_noalloc_equals_select_twice_shrinking():
    dev = device()
    big = wl.plain_instance("large", 1)                 # 2N = 20000, about 49 MiB of scratch
    small = wl.plain_instance("large", 2, M=3001)       # ragged, smaller, after the big one
    for inst in (big, small):
        ref, got, st = _both(inst, dev)
        assert st == nsga3.OK
        for k in KEYS:
            assert np.array_equal(got[k], ref[k]), k


def test_noalloc_many_objectives_and_status():
    dev = device()
    inst = wl.plain_instance("many_objective", 0, M=4000)
    ref, got, st = _both(inst, dev)
    assert st == nsga3.OK
    for k in KEYS:
        assert np.array_equal(got[k], ref[k]), k
    # a non-finite objective is reported through the status output
    F = inst["F"].copy()
    F[7, 1] = np.nan
    _, st2 = nsga3.select_noalloc(to_dev(F, dev), to_dev(inst["Z"], dev), inst["N"], 0)
    assert int(to_np(st2)[0]) == nsga3.ENONFINITE


def test_noalloc_rejects_beyond_scratch():
    dev = device()
    F = torch.zeros((30000, 3), dtype=torch.float32, device=dev)
    Z = torch.ones((5, 3), dtype=torch.float32, device=dev)
    with pytest.raises(nsga3.Nsga3Error) as e:
        nsga3.select_noalloc(F, Z, 15000, 0)
    assert e.value.code == nsga3.EWORKSPACE
