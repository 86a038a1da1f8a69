"""Test-only models of the niching step (Algorithm 1, niche-selection loop),
written independently of the oracle: a closed-form level ("water-fill")
formulation and an exhaustive enumeration of NSGA-III's random choices."""
from collections import defaultdict
from fractions import Fraction

import numpy as np

MASK = 2**64 - 1


def sm64(x):
    z = (x + 0x9E3779B97F4A7C15) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def key(seed, tag, j, L):
    return sm64((seed & MASK) ^ sm64((tag << 62) | (L << 32) | j))


def split(rank, fi, pi, H):
    l, S, K = int(fi[0]), int(fi[1]), int(fi[2])
    rho = np.zeros(H, np.int64)
    members = defaultdict(list)
    base = []
    for x in range(len(rank)):
        if rank[x] < l:
            rho[pi[x]] += 1
            base.append(x)
        elif rank[x] == l:
            members[int(pi[x])].append(x)
    return l, K, rho, members, base


def waterfill(rank, fi, pi, dist, H, seed):
    """Every reference is filled level by level: find the last complete level
    L*, give one more pick at L* to the first r references in key order, then
    make each reference's picks on its own."""
    l, K, rho, members, base = split(rank, fi, pi, H)
    c = np.zeros(H, np.int64)
    for j, v in members.items():
        c[j] = len(v)

    def P(L):
        return int(np.minimum(c, np.maximum(0, L - rho)).sum())

    if K >= c.sum():
        t = c.copy()
    else:
        L = 0
        while P(L + 1) <= K:
            L += 1
        r = K - P(L)
        T = [j for j in range(H) if c[j] > 0 and rho[j] <= L < rho[j] + c[j]]
        T.sort(key=lambda j: (key(seed, 1, j, L), j))
        t = np.minimum(c, np.maximum(0, L - rho))
        for j in T[:r]:
            t[j] += 1
    picks = []
    for j, mem in members.items():
        rem = sorted(mem)
        for lev in range(int(rho[j]), int(rho[j] + t[j])):
            if lev == 0:
                pos = min(range(len(rem)), key=lambda a: (dist[rem[a]], rem[a]))
            else:
                pos = key(seed, 2, j, lev) % len(rem)
            picks.append(rem.pop(pos))
    return np.array(sorted(base + picks), np.int32)


def enumerate_outcomes(rank, fi, pi, dist, H):
    """Distribution over selected sets of NSGA-III niching with uniform random
    choices: a reference uniformly among the least-crowded ones that still have
    candidates, then the nearest member at niche count 0, else a member
    uniformly at random."""
    l, K, rho0, members0, base = split(rank, fi, pi, H)
    out = defaultdict(Fraction)

    def rec(rho, mem, picked, prob):
        if len(picked) == K:
            out[tuple(sorted(base + picked))] += prob
            return
        act = [j for j in mem if mem[j]]
        L = min(rho[j] for j in act)
        V = [j for j in act if rho[j] == L]
        for v in V:
            if L == 0:
                choices = [min(mem[v], key=lambda x: (dist[x], x))]
            else:
                choices = list(mem[v])
            for x in choices:
                m2 = {j: list(a) for j, a in mem.items()}
                m2[v].remove(x)
                r2 = dict(rho)
                r2[v] += 1
                rec(r2, m2, picked + [x], prob / len(V) / len(choices))

    rec({j: int(rho0[j]) for j in range(H)}, {j: sorted(v) for j, v in members0.items()}, [], Fraction(1))
    return out
