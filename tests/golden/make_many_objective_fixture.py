"""Writes many_objective_seed0.txt: the FP64 oracle's full selection of the
many-objective workload (2N = 131072 merged points, m = 10, H = 2002
Das-Dennis references with p = 5, N = 65536, radius law 1 + U(0,1)^3,
seed 0), run once on the CPU.

Only the oracle (and the seeded input generator, which computes nothing of
the method) is called here. The oracle's sort at this size takes about a
minute with 8 threads (python tests/golden/make_many_objective_fixture.py).

The file holds front_info, the rank-0 membership bitmap (every ranked point
is in front 0 at this workload, so the bitmap is the whole rank vector), the
bitmap of the selected points, and SHA-256 digests of the oracle's
association (pi as little-endian int32 over all M points, -1 outside S_t).
Bitmaps are numpy packbits with little bit order, as hex, 64 bytes a line."""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2504_06067_amd import workloads as wl  # noqa: E402

OUT = os.path.join(HERE, "many_objective_seed0.txt")


def hexlines(bits):
    raw = np.packbits(bits.astype(np.uint8), bitorder="little").tobytes()
    return [raw[i:i + 64].hex() for i in range(0, len(raw), 64)]


def main():
    inst = wl.plain_instance("many_objective", 0)
    F, Z, N, seed = inst["F"], inst["Z"], inst["N"], inst["seed"]
    oracle.set_threads(int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1)))
    t0 = time.time()
    ref = oracle.select(F, Z, N, seed)
    print(f"oracle selection {time.time() - t0:.1f} s", flush=True)
    rank = ref["rank"]
    ranked = rank != oracle.UNRANKED
    assert np.all(rank[ranked] == 0), "the fixture format assumes a single ranked front"
    fi = (0, 0, N, 1)
    sel = np.zeros(len(F), bool)
    sel[ref["selected"]] = True
    pi_digest = hashlib.sha256(ref["pi"].astype("<i4").tobytes()).hexdigest()
    lines = [
        "# FP64 oracle selection of the many-objective workload: 2N=131072, m=10,",
        "# H=2002 (Das-Dennis p=5), N=65536, radius 1+U(0,1)^3, data seed 0, tie seed 0.",
        "# Written by tests/golden/make_many_objective_fixture.py (oracle only).",
        f"M {len(F)}",
        f"front_info {' '.join(str(v) for v in fi)}",
        f"ranked {int(ranked.sum())}",
        f"pi_sha256 {pi_digest}",
        "rank0_bitmap",
        *hexlines(ranked),
        "selected_bitmap",
        *hexlines(sel),
    ]
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
