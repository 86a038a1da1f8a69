"""Seeded synthetic inputs for the selection workloads.

Objective sets and reference sets only: nothing here computes any part of the
selection. Both the GPU path and the CPU oracle consume these arrays.

Objective laws (minimization, values in float32, drawn in float64 first):
a direction u = |z| / ||z|| with z ~ N(0, I_m) on the positive unit-sphere
orthant, scaled by a radius r >= 1 whose law depends on the workload.

Reference sets are Das-Dennis simplex lattices: every composition
(c_1, ..., c_m) of p into m non-negative parts, in lexicographically
ascending order, mapped to c / p. Their count is C(p + m - 1, m - 1).
"""
import math

import numpy as np


def das_dennis_counts(m, p):
    """Integer compositions of p into m parts, lexicographically ascending."""
    out = []
    cur = [0] * m

    def rec(pos, left):
        if pos == m - 1:
            cur[pos] = left
            out.append(tuple(cur))
            return
        for c in range(left + 1):
            cur[pos] = c
            rec(pos + 1, left - c)

    rec(0, p)
    return np.array(out, dtype=np.int64).reshape(-1, m)


def das_dennis(m, p):
    """Single-layer reference set, float32 [H][m]."""
    c = das_dennis_counts(m, p)
    return (c.astype(np.float64) / p).astype(np.float32)


def das_dennis_two_layer(m, p1, p2):
    """Boundary layer (p1) followed by an inner layer (p2) shrunk towards the
    simplex centre: w' = w / 2 + 1 / (2 m)."""
    outer = das_dennis_counts(m, p1).astype(np.float64) / p1
    inner = das_dennis_counts(m, p2).astype(np.float64) / p2
    inner = inner / 2.0 + 1.0 / (2.0 * m)
    return np.concatenate([outer, inner]).astype(np.float32)


def ref_count(m, p):
    return math.comb(p + m - 1, m - 1)


def directions(rng, M, m):
    z = np.abs(rng.standard_normal((M, m)))
    return z / np.linalg.norm(z, axis=1, keepdims=True)


def objectives(rng, M, m, law):
    """float32 [M][m] objective vectors under one of the radius laws."""
    u = directions(rng, M, m)
    if law == "sphere_half":          # half on the unit sphere, half at 1 + U(0, 0.5)
        r = np.ones(M)
        h = M // 2
        r[h:] = 1.0 + rng.uniform(0.0, 0.5, M - h)
    elif law == "exp":                # 1 + g, g ~ Exponential(scale 0.3): many fronts
        r = 1.0 + rng.exponential(0.3, M)
    elif law == "cube":               # 1 + U(0,1)^3: few dominance relations
        r = 1.0 + rng.uniform(0.0, 1.0, M) ** 3
    else:
        raise ValueError(law)
    return (u * r[:, None]).astype(np.float32)


# The plain workloads: (2N, m, p, law).
PLAIN = {
    "small": dict(M=184, m=3, p=12, law="sphere_half"),
    "large": dict(M=20000, m=3, p=140, law="exp"),
    "many_objective": dict(M=131072, m=10, p=5, law="cube"),
}


def plain_instance(name, seed=0, M=None):
    """One plain selection instance: F [M][m], Z [H][m], N = M / 2, seed.
    M may be overridden (even) to draw a smaller instance of the same law."""
    cfg = PLAIN[name]
    M = cfg["M"] if M is None else int(M)
    rng = np.random.default_rng(seed)
    F = objectives(rng, M, cfg["m"], cfg["law"])
    Z = das_dennis(cfg["m"], cfg["p"])
    return dict(name=name, F=F, Z=Z, M=M, m=cfg["m"], H=Z.shape[0], N=M // 2, seed=seed)


BATCH_M = (3, 5, 8, 10)
BATCH_P = {3: 40, 5: 8, 8: 4, 10: 3}


def batched_instances(seed=0, count=64, lo=2000, hi=40000):
    """Independent instances of uneven size: 2N log-uniform in [lo, hi] (even),
    m uniform over {3, 5, 8, 10} with Das-Dennis p of {40, 8, 4, 3}; objectives
    follow the exponential-radius law; instance b uses data seed seed*1000+b."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        M = 2 * int(round(math.exp(rng.uniform(math.log(lo), math.log(hi))) / 2))
        m = int(BATCH_M[rng.integers(len(BATCH_M))])
        r2 = np.random.default_rng(seed * 1000 + b)
        F = objectives(r2, M, m, "exp")
        Z = das_dennis(m, BATCH_P[m])
        out.append(dict(F=F, Z=Z, M=M, m=m, H=Z.shape[0], N=M // 2, seed=seed * 1000 + b))
    return out


def random_small(rng, M, m, kind="continuous"):
    """Small adversarial objective sets for exhaustive checks: continuous
    values, coarse integer grids (many ties and duplicates), or chains."""
    if kind == "continuous":
        return rng.random((M, m)).astype(np.float32)
    if kind == "grid":
        return rng.integers(0, 4, (M, m)).astype(np.float32)
    if kind == "chain":
        t = rng.permutation(M).astype(np.float32)
        return np.repeat(t[:, None], m, axis=1)
    if kind == "equal":
        return np.ones((M, m), np.float32)
    raise ValueError(kind)


# Served requests: m -> reference set (single layer p, or two layers (p1, p2)).
SERVED_REFS = {3: (40,), 5: (8,), 10: (3,), 15: (2, 1)}
SERVED_D = 12
SERVED_GENERATIONS = 50


def served_refs(m):
    p = SERVED_REFS[m]
    return das_dennis(m, p[0]) if len(p) == 1 else das_dennis_two_layer(m, p[0], p[1])


def served_trace(seed=0, count=256, qps=1.0, lo=1000, hi=100000, ms=(3, 5, 10, 15),
                 d=SERVED_D, generations=SERVED_GENERATIONS):
    """Request stream: Poisson arrivals at rate `qps` (seconds), 2N
    log-uniform in [lo, hi] (even), m uniform over `ms`; each request carries
    its reference set, a seeded N(0, 1) objective-map matrix A [m][d-1] and
    its own seed. Arrival times are returned relative to the first (0)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / qps, count)
    t = np.concatenate([[0.0], np.cumsum(gaps[1:])])
    out = []
    for r in range(count):
        M = 2 * int(round(math.exp(rng.uniform(math.log(lo), math.log(hi))) / 2))
        m = int(ms[rng.integers(len(ms))])
        ra = np.random.default_rng(seed * 100003 + r)
        A = ra.standard_normal((m, d - 1)).astype(np.float32)
        out.append(dict(rid=r, arrival=float(t[r]), M=M, N=M // 2, m=m, d=d, Z=served_refs(m),
                        A=A, generations=generations, seed=seed * 1000003 + r))
    return out
