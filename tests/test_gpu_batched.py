"""Batched selection: every instance of a batch gets exactly what a plain
nsga3_select on the same arguments gives (bit for bit, all intermediates),
whatever the batch around it and whatever its tile parameters; the plain
results are in turn checked against the oracle. Also: graph capture and
replay of a batched call, and per-instance status words."""
import numpy as np
import pytest
import torch

from gpu_util import device, select_parity, to_dev, to_np
from paper_2504_06067_amd import nsga3
from paper_2504_06067_amd import workloads as wl

pytestmark = pytest.mark.gpu

KEYS = ("selected", "rank", "pi", "dist")


def mixed_instances(seed, count, lo=100, hi=6000):
    """Uneven small instances over several m (and laws), oracle-sized."""
    rng = np.random.default_rng(seed)
    laws = ("exp", "cube", "sphere_half")
    mp = {2: 60, 3: 12, 5: 5, 8: 3, 10: 3}
    out = []
    for b in range(count):
        M = 2 * int(round(np.exp(rng.uniform(np.log(lo), np.log(hi))) / 2))
        m = int(list(mp)[rng.integers(len(mp))])
        F = wl.objectives(np.random.default_rng(seed * 100 + b), M, m, laws[b % 3])
        Z = wl.das_dennis(m, mp[m])
        N = int(rng.integers(1, M + 1)) if b % 4 == 3 else M // 2
        out.append(dict(F=F, Z=Z, M=M, m=m, H=len(Z), N=N, seed=seed * 100 + b))
    return out


def as_problems(insts, dev, tiles=None):
    probs = []
    for b, q in enumerate(insts):
        p = dict(F=to_dev(q["F"], dev), Z=to_dev(q["Z"], dev), N=q["N"], seed=q["seed"])
        if tiles is not None:
            p["tile"] = tiles[b]
        probs.append(p)
    return probs


def run_batched(insts, dev, tiles=None):
    bt = nsga3.Batch(as_problems(insts, dev, tiles), intermediates=True)
    bt.run()
    torch.cuda.synchronize()
    assert bt.status() == [nsga3.OK] * len(insts)
    return [{k: to_np(getattr(bt, k)[b]) for k in KEYS} for b in range(len(insts))]


def run_plain(q, dev):
    out = nsga3.select(to_dev(q["F"], dev), to_dev(q["Z"], dev), q["N"], q["seed"],
                       intermediates=True)
    return {k: to_np(v) for k, v in out.items()}


def same(a, b):
    return all(np.array_equal(a[k], b[k]) for k in KEYS)


def check_oracle(q, g, dev):
    """The FP64 oracle's bar for a batched result (see select_parity)."""
    r = select_parity(q, g, dev)
    assert r["ext_ties"] == 0
    assert r["pi_ties"] <= max(2, 1e-3 * r["n_st"])
    return r


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_batched_equals_plain_and_oracle(seed):
    dev = device()
    insts = mixed_instances(seed, 12)
    got = run_batched(insts, dev)
    for q, g in zip(insts, got):
        assert same(g, run_plain(q, dev)), (q["M"], q["m"], q["N"])
        check_oracle(q, g, dev)


def test_tile_invariance():
    dev = device()
    insts = mixed_instances(7, 8)
    base = run_batched(insts, dev)
    def slice_of(H, r):
        if r == "H":
            return H
        return r if r <= H else H

    for g_tile, r_tile in [(1, 16), (3, 0), (64, 32), (1000, "H"), (1 << 30, 48)]:
        tiles = [[g_tile, slice_of(q["H"], r_tile), 0, 0] for q in insts]
        got = run_batched(insts, dev, tiles)
        for a, b in zip(base, got):
            assert same(a, b), (g_tile, r_tile)
    # the autotuned table's tiles (dominance items and association slices)
    from paper_2504_06067_amd import autotune
    tuned = [autotune.lookup(q["M"], q["m"], q["H"]) for q in insts]
    got = run_batched(insts, dev, tuned)
    for a, b in zip(base, got):
        assert same(a, b), "tuned tiles"


def test_alone_equals_in_mix():
    dev = device()
    insts = mixed_instances(11, 10)
    mix = run_batched(insts, dev)
    for b in (0, 4, 9):
        alone = run_batched([insts[b]], dev)[0]
        assert same(alone, mix[b])
    # and in another order
    perm = [9, 3, 0, 7, 1, 8, 2, 6, 4, 5]
    shuffled = run_batched([insts[i] for i in perm], dev)
    for pos, i in enumerate(perm):
        assert same(shuffled[pos], mix[i])


def test_uneven_batch_full_size():
    """The 64-instance uneven workload at full size: each instance equals its
    plain run; the smallest few are also checked against the oracle."""
    dev = device()
    insts = wl.batched_instances(0, 64)
    got = run_batched(insts, dev)
    for q, g in zip(insts, got):
        assert same(g, run_plain(q, dev)), (q["M"], q["m"])
    for b in sorted(range(64), key=lambda i: insts[i]["M"])[:3]:
        check_oracle(insts[b], got[b], dev)


def test_streamed_peel_repeated():
    """Large multi-front instances whose peel streams matrix columns (more
    chunks than the register caches hold), so that workgroups own several
    chunks of one instance: every call of the batch, and every call of the
    plain path, gives the same ranks and selection."""
    dev = device()
    shapes = [(79048, 3), (85532, 5), (60000, 10), (45000, 15), (70000, 3)]
    probs = []
    for i, (M, m) in enumerate(shapes):
        F = to_dev(wl.objectives(np.random.default_rng(M), M, m, "exp"), dev)
        Z = to_dev(wl.served_refs(m), dev)
        probs.append(dict(F=F, Z=Z, N=M // 2, seed=11 + i))
    plain = []
    for p in probs:
        o = nsga3.select(p["F"], p["Z"], p["N"], p["seed"], intermediates=True)
        plain.append({k: to_np(o[k]).copy() for k in ("selected", "rank")})
    bt = nsga3.Batch(probs, intermediates=True)
    for call in range(24):
        bt.run()
        torch.cuda.synchronize()
        assert bt.status() == [nsga3.OK] * len(probs), call
        for b in range(len(probs)):
            assert np.array_equal(to_np(bt.rank[b]), plain[b]["rank"]), (call, b)
            assert np.array_equal(to_np(bt.selected[b]), plain[b]["selected"]), (call, b)
    p = probs[0]
    for call in range(8):
        o = nsga3.select(p["F"], p["Z"], p["N"], p["seed"], intermediates=True)
        assert np.array_equal(to_np(o["rank"]), plain[0]["rank"]), call


def test_graph_replay():
    dev = device()
    insts = mixed_instances(5, 6)
    bt = nsga3.Batch(as_problems(insts, dev), intermediates=True)
    bt.run()
    torch.cuda.synchronize()
    eager = [{k: to_np(getattr(bt, k)[b]).copy() for k in KEYS} for b in range(len(insts))]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        bt.run()  # warm-up on the side stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        bt.run()
    for rep in range(4):
        for b in range(len(insts)):
            bt.selected[b].fill_(-7)
            bt.rank[b].fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for b in range(len(insts)):
            got = {k: to_np(getattr(bt, k)[b]) for k in KEYS}
            assert same(got, eager[b]), (rep, b)
        # eager work between replays
        bt.run()
        torch.cuda.synchronize()
    assert bt.status() == [nsga3.OK] * len(insts)


def test_status_per_instance():
    dev = device()
    insts = mixed_instances(3, 4)
    bad = dict(insts[2])
    F = bad["F"].copy()
    F[5, 1] = np.nan
    bad["F"] = F
    insts[2] = bad
    bt = nsga3.Batch(as_problems(insts, dev))
    bt.run()
    st = bt.status()
    assert st[2] == nsga3.ENONFINITE
    assert st[0] == st[1] == st[3] == nsga3.OK


def test_batched_rejects_bad_arguments():
    dev = device()
    insts = mixed_instances(4, 2)
    for tile in ([(1 << 30) + 1, 0, 0, 0], [0, 7, 0, 0], [0, 0, 1, 0], [-1, 0, 0, 0]):
        with pytest.raises(nsga3.Nsga3Error):
            nsga3.Batch(as_problems(insts, dev, [tile, [0, 0, 0, 0]]))
    bt = nsga3.Batch(as_problems(insts, dev))
    small = bt.buf[: bt.buf.numel() // 2]
    rc = nsga3.lib().nsga3_select_batched(bt.arr, bt.B, nsga3._ptr(small), small.numel(),
                                          nsga3._stream(dev))
    assert rc == nsga3.EWORKSPACE


def _instances_of_m(ms, seed, M=1200):
    out = []
    for b, m in enumerate(ms):
        rng = np.random.default_rng(seed * 100 + b)
        F = wl.objectives(rng, M + 64 * b, m, "exp")
        p = {2: 60, 3: 12, 4: 6, 5: 5, 6: 4, 7: 3, 8: 3, 9: 3, 10: 3, 11: 2}.get(m, 1)
        Z = wl.das_dennis(m, p)
        out.append(dict(F=F, Z=Z, M=len(F), m=m, H=len(Z), N=len(F) // 2, seed=seed * 100 + b))
    return out


@pytest.mark.parametrize("ms", [
    [3, 20, 5, 20, 3],                 # a group with m > 16: peels pipelined, the
                                       # normalization and association on the caller's stream
    [2, 3, 4, 5, 6, 7, 8, 9, 10, 11],  # more m-groups than the pipeline takes: one peel
    [5, 3],                            # two groups
])
def test_group_layouts_equal_plain(ms):
    """Every way the batched call schedules its m-groups gives each instance
    exactly its plain result."""
    dev = device()
    insts = _instances_of_m(ms, 21)
    got = run_batched(insts, dev)
    for q, g in zip(insts, got):
        assert same(g, run_plain(q, dev)), (q["M"], q["m"])
