"""Autotuner for the per-instance tile parameters of batched selection.

Two parameters shape the work split without changing any result:
  tile[0]  dominance tiles per work item; 0 lets the library size items from
           the tiles of the whole launch (all instances of equal m)
  tile[1]  references per association slice (a multiple of 16, or H)
For every (m, size class) bucket the tuner times, on a synthetic instance of
that shape (the large workload's radius law) and with HIP events around the
kernel, each slice width for the association and then each item size for the
dominance kernel. It keeps the fastest slice width, and an explicit item
size only when it beats the library's launch-wide choice by more than
G_MARGIN (that choice also serves mixed launches, which one instance's
timing does not see). The table is JSON, keyed "m:log2(2N)"; ``lookup``
returns the tiles for an instance, or zeros (the library's own choice) when
its bucket was not tuned.

Usage (on the GPU):  python -m paper_2504_06067_amd.autotune --out tiles.json
"""
import argparse
import json
import math
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
TABLE_PATH = os.path.join(_HERE, "tiles.json")

R_CANDIDATES = (32, 64, 128, 256, 512)
G_CANDIDATES = (1, 2, 3, 4, 6, 12)
G_MARGIN = 0.02

_table = None


def bucket(M, m):
    return f"{int(m)}:{max(8, int(round(math.log2(max(int(M), 2)))))}"


def load(path=TABLE_PATH):
    global _table
    if _table is None:
        _table = {}
        if os.path.exists(path):
            with open(path) as f:
                _table = json.load(f).get("tiles", {})
    return _table


def lookup(M, m, H):
    """[G, R, 0, 0] for an instance of 2N = M, m objectives, H references."""
    t = load().get(bucket(M, m))
    if not t:
        return [0, 0, 0, 0]
    G, R = int(t[0]), int(t[1])
    if R >= H:
        R = H
    elif R % 16:
        R = 0
    return [G, R, 0, 0]


def _time_kernel(bt, names, reps):
    import torch

    from . import nsga3

    for _ in range(2):
        bt.run()
    torch.cuda.synchronize()
    nsga3.profile_enable(",".join(names))
    for _ in range(reps):
        bt.run()
    torch.cuda.synchronize()
    out = {}
    for n in names:
        tot, _, _ = nsga3.profile_read(n)
        out[n] = tot / reps * 1e3  # microseconds per call, all launches of the kernel
    nsga3.profile_enable(None)
    return out


def tune(buckets, device="cuda:0", reps=5, seed=0, log=print):
    """buckets: iterable of (M, m, p). Returns the table dict."""
    import numpy as np
    import torch

    from . import nsga3, workloads

    dev = torch.device(device)
    table = {}
    for M, m, p in buckets:
        rng = np.random.default_rng(seed)
        F = torch.from_numpy(workloads.objectives(rng, M, m, "exp")).to(dev)
        Zn = workloads.das_dennis(m, p)
        Z = torch.from_numpy(Zn).to(dev)
        H = len(Zn)
        base = dict(F=F, Z=Z, N=M // 2, seed=seed)
        best_r, best_rt = 0, float("inf")
        for R in R_CANDIDATES + (H,):
            if R > H or (R != H and R % 16):
                continue
            bt = nsga3.Batch([dict(base, tile=[0, R, 0, 0])])
            t = _time_kernel(bt, ["associate"], reps)["associate"]
            if t < best_rt:
                best_r, best_rt = R, t
        auto_t = _time_kernel(nsga3.Batch([dict(base, tile=[0, best_r, 0, 0])]), ["dominance"],
                              reps)["dominance"]
        best_g, best_gt = 0, auto_t
        for G in G_CANDIDATES:
            bt = nsga3.Batch([dict(base, tile=[G, best_r, 0, 0])])
            t = _time_kernel(bt, ["dominance"], reps)["dominance"]
            if t < best_gt and t < auto_t * (1.0 - G_MARGIN):
                best_g, best_gt = G, t
        key = bucket(M, m)
        table[key] = [best_g, best_r]
        log(f"{key} (2N={M}, H={H}): R={best_r} ({best_rt:.1f} us), G={best_g} "
            f"({best_gt:.1f} us against {auto_t:.1f} us for the launch-wide choice)")
        del F, Z
    return table


DEFAULT_BUCKETS = [(M, m, p) for m, p in ((3, 40), (5, 8), (8, 4), (10, 3), (15, 2))
                   for M in (2048, 4096, 8192, 16384, 32768, 65536, 131072)]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TABLE_PATH)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    table = tune(DEFAULT_BUCKETS, reps=args.reps)
    with open(args.out, "w") as f:
        json.dump({"note": "tiles per bucket m:round(log2(2N)) = [dominance tiles per work "
                           "item (0: the library sizes them from the whole launch; an "
                           "explicit size only where it was more than 2 % faster), "
                           "references per association slice]; written by "
                           "python -m paper_2504_06067_amd.autotune",
                   "tiles": table}, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
