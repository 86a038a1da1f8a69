"""Readers of the stored fixtures under tests/golden/ (values written by
oracle-only scripts that sit beside them)."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _bits(hexlines, M):
    raw = bytes.fromhex("".join(hexlines))
    return np.unpackbits(np.frombuffer(raw, np.uint8), bitorder="little")[:M].astype(bool)


def many_objective_seed0():
    """dict(M, front_info, ranked (bool[M]), selected (int32 ascending),
    pi_sha256) of the oracle's full selection of the many-objective
    workload at seed 0 (make_many_objective_fixture.py)."""
    with open(os.path.join(GOLDEN, "many_objective_seed0.txt")) as f:
        lines = [ln.strip() for ln in f if ln.strip() and not ln.startswith("#")]
    out = {}
    i = 0
    while i < len(lines):
        key, _, val = lines[i].partition(" ")
        if key in ("rank0_bitmap", "selected_bitmap"):
            j = i + 1
            while j < len(lines) and not lines[j].endswith("_bitmap"):
                j += 1
            out[key] = lines[i + 1:j]
            i = j
            continue
        out[key] = val
        i += 1
    M = int(out["M"])
    return dict(M=M, front_info=np.array([int(v) for v in out["front_info"].split()], np.int32),
                ranked=_bits(out["rank0_bitmap"], M),
                selected=np.where(_bits(out["selected_bitmap"], M))[0].astype(np.int32),
                n_ranked=int(out["ranked"]), pi_sha256=out["pi_sha256"])
