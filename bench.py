"""Benchmark: NSGA-III environmental selection on one MI355X.

A step is one nsga3_select (non-dominated sort -> normalization ->
association -> niching) over the plain large workload: 2N = 20000 merged
float32 objective vectors, m = 3, H = 10011 Das-Dennis references (p = 140),
N = 10000 survivors, radius law 1 + Exponential(scale 0.3). Inputs are
resident in HBM before the timed region. The JSON line reports

  value           merged solutions selected per second (2N * steps / wall time)
  latency_ms      p50 / p99 of the per-step time (HIP events on the stream)
  roofline        the dominant kernel (dominance matrix) against the VALU issue
                  peak, its time measured with HIP events inside the timed loop
  kernels         per-kernel times of a separate profiled pass; association
                  against the VALU issue peak, the peel's matrix reads against
                  HBM
  small           2N = 184 (m = 3, H = 91): p50 / p99 over 2000 selections
  many_objective  2N = 131072 (m = 10, H = 2002): p50 / p99, dominance fraction
  generation_loop whole generations (evolve + select) at the Table I shapes
  objective_scaling  selection at 2N = 1600, m = 4..512 (Table II shapes)
  batched         64 uneven instances, one graph replay vs 64 plain calls
  served          continuous batching vs the one-at-a-time plain loop on the
                  same Poisson trace, per offered load
  niche_ab        the niche stage alone: the closed form against the paper's
                  cache-tensor loop, on each workload's own GPU intermediates
  cpu_baseline    the FP64 CPU oracle on a bounded sample of the same workload,
                  single-threaded and on all usable cores
  parity          per workload, from the oracle run in the CPU-baseline leg:
                  near-tie counts and the FP64 distance error of the GPU's
                  association

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "merged solutions selected/sec + p50/p99 latency, batched/served vs plain"
# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz, one lane-op per lane per clock
VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="large", choices=["small", "large", "many_objective"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-reps", type=int, default=20)
    ap.add_argument("--batched-no-plain", action="store_true",
                    help="batched leg: graph replays only (no plain comparison), for profiling")
    ap.add_argument("--only-batched", action="store_true",
                    help="run the batched comparison alone (for profiling it separately)")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run one device-to-device copy of this size first (the reference "
                         "kernel that scales HBM counters in a --pmc run)")
    ap.add_argument("--only-served", action="store_true",
                    help="run the served comparison alone (for profiling it separately)")
    ap.add_argument("--served-requests", type=int, default=256)
    ap.add_argument("--served-generations", type=int, default=50)
    ap.add_argument("--served-budget-gb", type=float, default=64.0)
    ap.add_argument("--no-niche-ab", action="store_true",
                    help="skip the niche-stage A/B (closed form against the cache-tensor loop)")
    ap.add_argument("--served-loads", default="0.5,1,2,4",
                    help="offered loads, comma-separated fractions of the plain loop's capacity "
                         "(e.g. 0.5,1,2,4 for the sweep)")
    ap.add_argument("--cpu-seconds", type=float, default=8.0,
                    help="target CPU time of each oracle sample (single thread, all cores)")
    ap.add_argument("--no-kernels", action="store_true",
                    help="skip the per-kernel profiled pass")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the small and many-objective latency legs")
    ap.add_argument("--small-reps", type=int, default=2000)
    ap.add_argument("--no-objective-scaling", action="store_true",
                    help="skip the selection at m = 4..512 (Table II shapes)")
    ap.add_argument("--no-generations", action="store_true",
                    help="skip the whole-generation loop at the Table I shapes")
    ap.add_argument("--many-reps", type=int, default=20)
    return ap.parse_args()


def host_cpu():
    """CPU model, logical CPUs, and the CPUs this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, os.cpu_count() or 1, usable


def _time_oracle(inst, target_s, threads):
    import oracle

    oracle.set_threads(threads)
    try:
        t0 = time.perf_counter()
        oracle.select(inst["F"], inst["Z"], inst["N"], inst["seed"])
        first = time.perf_counter() - t0
        reps = max(1, min(20, int(math.floor(target_s / max(first, 1e-9)))) - 1)
        t0 = time.perf_counter()
        for _ in range(reps):
            oracle.select(inst["F"], inst["Z"], inst["N"], inst["seed"])
        el = time.perf_counter() - t0 if reps else first
    finally:
        oracle.set_threads(1)
    n = reps if reps else 1
    return inst["M"] * n / el, n, el


def cpu_baseline(inst, target_s):
    """The oracle, as it stands, on full selections of the same instance:
    single-threaded (the reported value) and with its dominance and
    association loops on all usable host cores (at most 16, the box's share
    of one GPU)."""
    model, nproc, usable = host_cpu()
    v1, n1, el1 = _time_oracle(inst, target_s, 1)
    threads = max(1, min(usable, 16))
    vn, nn, eln = _time_oracle(inst, target_s, threads)
    return {
        "value": v1,
        "unit": "merged solutions/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{n1} full selection(s) of the same instance (2N={inst['M']}, m={inst['m']}, "
                  f"H={inst['H']}) after one untimed run; {el1:.1f} s single-threaded FP64 C",
        "all_cores": {"value": vn, "unit": "merged solutions/s", "cores": threads,
                      "sample": f"{nn} full selection(s), {eln:.1f} s, OpenMP over the dominance "
                                f"and association loops"},
        "cpu_model": model,
        "nproc": nproc,
        "usable_cpus": usable,
    }


def parity_report(dev, gpu_out, inst, threads):
    """The near-tie counts and the distance error of one GPU selection against
    the FP64 oracle's normalization and association at the GPU's ranks (ranks
    themselves are checked bit for bit by the test-suite): extreme points
    whose FP64 ASF gap is within 1e-6 relative, association mismatches whose
    FP64 distance gap is within 1e-6 ||f_n|| (any other mismatch is an
    error), max |d_gpu - d_oracle| / ||f_n||, and whether the selection equals
    the oracle's niching of the GPU's own (rank, pi, dist)."""
    import numpy as np
    import oracle

    from paper_2504_06067_amd import nsga3

    F, Z, N, seed = inst["F"], inst["Z"], inst["N"], inst["seed"]
    g = {k: v.cpu().numpy() for k, v in gpu_out.items()}
    rank = g["rank"]
    ranked = rank[rank != nsga3.UNRANKED]
    l = int(ranked.max())
    S = int(np.sum(ranked < l))
    fi = np.array([l, S, N - S, l + 1], np.int32)
    oracle.set_threads(threads)
    try:
        nrm = oracle.normalize(F, rank, fi)
        pi_ref, d_ref = oracle.associate(nrm["Fn"], rank, fi, Z)
    finally:
        oracle.set_threads(1)
    import torch
    ext = nsga3.normalize(torch.from_numpy(F).to(dev), gpu_out["rank"],
                          torch.from_numpy(fi).to(dev))["extreme"].cpu().numpy()
    z = nrm["ideal"]
    ext_ties = 0
    for k in range(F.shape[1]):
        if ext[k] != nrm["extreme"][k]:
            def asf(x):
                fp = F[x].astype(np.float64) - z
                v = 1e6 * fp
                v[k] = fp[k]
                return v.max()
            a, b = asf(ext[k]), asf(nrm["extreme"][k])
            if abs(a - b) > 1e-6 * max(abs(b), 1e-30):
                raise RuntimeError(f"extreme point {k} differs beyond the near-tie band")
            ext_ties += 1
    st = np.where(rank <= l)[0]
    Fn = np.nan_to_num(nrm["Fn"][st], nan=0.0)
    norms = np.maximum(np.linalg.norm(Fn, axis=1), 1e-30)
    derr = float(np.max(np.abs(g["dist"][st].astype(np.float64) - d_ref[st]) / norms))
    W = Z.astype(np.float64)
    W /= np.linalg.norm(W, axis=1, keepdims=True)

    def pdist(rows, refs):
        f = Fn[rows]
        w = W[refs]
        p = np.sum(f * w, axis=1, keepdims=True)
        return np.linalg.norm(f - p * w, axis=1)

    mis = np.where(g["pi"][st] != pi_ref[st])[0]
    gap = np.abs(pdist(mis, g["pi"][st][mis]) - pdist(mis, pi_ref[st][mis])) / norms[mis]
    pi_ties = int(np.sum(gap <= 1e-6))
    if ext_ties == 0 and pi_ties != len(mis):
        raise RuntimeError(f"{len(mis) - pi_ties} association mismatches beyond the near-tie band")
    chained = oracle.niche(rank, fi, g["pi"], g["dist"].astype(np.float64), len(Z), N, seed)
    return {"points_in_S_t": int(len(st)), "extreme_near_ties": ext_ties,
            "assoc_near_ties": pi_ties, "assoc_mismatches": int(len(mis)),
            "dist_err_max_rel_fn": derr,
            "selection_equals_oracle_niching": bool(np.array_equal(g["selected"], chained))}


def _median_ms(fn, reps, stream):
    import numpy as np
    import torch

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    t = np.array([a.elapsed_time(b) for a, b in ev])
    return float(np.median(t)), float(np.percentile(t, 99))


def bench_batched(args, dev):
    """64 uneven instances: one graph replay of the batched call against the
    same 64 instances as back-to-back plain calls (with and without a host
    sync after each). Throughput counts merged solutions of all instances."""
    import torch

    from paper_2504_06067_amd import nsga3, workloads

    insts = workloads.batched_instances(args.seed, 64)
    total = sum(q["M"] for q in insts)
    probs = [dict(F=torch.from_numpy(q["F"]).to(dev), Z=torch.from_numpy(q["Z"]).to(dev),
                  N=q["N"], seed=q["seed"]) for q in insts]
    stream = torch.cuda.current_stream(dev)
    bt = nsga3.Batch(probs)
    for _ in range(3):
        bt.run()
    torch.cuda.synchronize()
    side = torch.cuda.Stream(dev)
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        bt.run()
    stream.wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        bt.run()
    graph.replay()
    torch.cuda.synchronize()
    if bt.status() != [nsga3.OK] * len(insts):
        raise RuntimeError("batched status not OK")
    g_med, g_p99 = _median_ms(graph.replay, args.batched_reps, stream)
    if args.batched_no_plain:
        # graph replays only (for a kernel trace of the batched call alone)
        return {"graph_ms": {"p50": g_med, "p99": g_p99}, "value": total / (g_med / 1e3)}
    e_med, _ = _median_ms(bt.run, args.batched_reps, stream)

    wss = [nsga3.Workspace(dev) for _ in probs]
    outs = [torch.empty(p["N"], dtype=torch.int32, device=dev) for p in probs]

    def plain():
        for p, w, o in zip(probs, wss, outs):
            nsga3.select(p["F"], p["Z"], p["N"], p["seed"], ws=w, out=o)

    def plain_sync():
        for p, w, o in zip(probs, wss, outs):
            nsga3.select(p["F"], p["Z"], p["N"], p["seed"], ws=w, out=o)
            torch.cuda.synchronize()

    plain()
    torch.cuda.synchronize()
    p_med, _ = _median_ms(plain, max(3, args.batched_reps // 2), stream)
    t0 = time.perf_counter()
    reps = max(3, args.batched_reps // 4)
    for _ in range(reps):
        plain_sync()
    ps_ms = (time.perf_counter() - t0) * 1e3 / reps
    for w in wss:
        if w.status() != nsga3.OK:
            raise RuntimeError("plain status not OK")
    return {
        "workload": "64 uneven instances, 2N log-uniform [2000, 40000], m in {3,5,8,10}, "
                    f"sum 2N = {total}",
        "graph_ms": {"p50": g_med, "p99": g_p99},
        "batched_eager_ms": e_med,
        "plain_back_to_back_ms": p_med,
        "plain_synced_ms": ps_ms,
        "value": total / (g_med / 1e3),
        "plain_value": total / (p_med / 1e3),
        "unit": "merged solutions/s",
        "speedup_vs_plain": p_med / g_med,
        "speedup_vs_plain_synced": ps_ms / g_med,
    }


def bench_served(args, dev):
    """Resident runs (50 generations each) arriving as a Poisson stream:
    the continuous-batching server against the plain loop that serves one
    request at a time with plain calls, on the same trace, at each offered
    load of --served-loads (fractions of the plain loop's capacity mu,
    measured first by running the requests back to back). Throughput is the
    merged solutions selected over the makespan; latency is arrival to
    result, p50/p99; every run's result must be identical in both modes."""
    import numpy as np

    from paper_2504_06067_amd import serve, workloads

    R, G = args.served_requests, args.served_generations
    budget = int(args.served_budget_gb * (1 << 30))
    calib = workloads.served_trace(args.seed, R, qps=1.0, generations=G)
    t_cal = serve.Server(dev, budget=budget, mode="plain").run(calib, realtime=False)
    mu = R / t_cal[None]["makespan_s"]
    points = []
    for load in [float(x) for x in args.served_loads.split(",")]:
        qps = load * mu
        trace = workloads.served_trace(args.seed, R, qps=qps, generations=G)
        work = sum(q["M"] * G for q in trace)
        out, results = {}, {}
        for mode in ("batched", "plain"):
            r = serve.Server(dev, budget=budget, mode=mode).run(trace, realtime=True)
            results[mode] = r
            lat = np.array([r[q["rid"]]["latency_s"] for q in trace])
            bad = [q["rid"] for q in trace if r[q["rid"]]["status"] != 0]
            if bad:
                raise RuntimeError(f"served status not OK for requests {bad[:5]}")
            span = r[None]["makespan_s"]
            out[mode] = {"latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                                        "p99": float(np.percentile(lat, 99) * 1e3),
                                        "mean": float(lat.mean() * 1e3)},
                         "makespan_s": span, "value": work / span, "ticks": r[None]["ticks"],
                         "peak_active": r[None]["peak_active"],
                         "bypasses": r[None]["bypasses"],
                         "peak_pool_gb": r[None]["peak_pool_bytes"] / (1 << 30)}
        same = all(np.array_equal(results["batched"][q["rid"]]["X"], results["plain"][q["rid"]]["X"])
                   and np.array_equal(results["batched"][q["rid"]]["F"],
                                      results["plain"][q["rid"]]["F"]) for q in trace)
        points.append({
            "load": load, "qps": qps,
            "arrivals_end_s": float(trace[-1]["arrival"]),
            "served": out["batched"], "plain": out["plain"],
            "throughput_ratio": out["batched"]["value"] / out["plain"]["value"],
            "speedup_p50": out["plain"]["latency_ms"]["p50"] / out["batched"]["latency_ms"]["p50"],
            "speedup_p99": out["plain"]["latency_ms"]["p99"] / out["batched"]["latency_ms"]["p99"],
            "results_identical": bool(same),
        })
        print(f"served load {load}: throughput x{points[-1]['throughput_ratio']:.2f}, "
              f"p50 x{points[-1]['speedup_p50']:.2f}, p99 x{points[-1]['speedup_p99']:.2f}",
              file=sys.stderr, flush=True)
    # headline: offered load 2 mu (above the plain loop's capacity, where
    # continuous batching can raise throughput); every load is in "sweep"
    first = next((p for p in points if p["load"] == 2.0), points[-1])
    quality = served_quality(dev, trace, results["batched"])
    return {
        "workload": f"{R} requests, Poisson arrivals, 2N log-uniform [1000, 100000], m in "
                    f"{{3,5,10,15}}, d=12, {G} generations each (SBX + polynomial mutation + "
                    f"synthetic objective map, then selection)",
        "unit": "merged solutions selected/s (sum of 2N x generations / makespan)",
        "plain_capacity_rps": mu,
        "hbm_budget_gb": args.served_budget_gb,
        "load": first["load"], "qps": first["qps"],
        "served": first["served"], "plain": first["plain"],
        "throughput_ratio": first["throughput_ratio"],
        "speedup_p50": first["speedup_p50"], "speedup_p99": first["speedup_p99"],
        "results_identical": all(p["results_identical"] for p in points),
        "sweep": points,
        "quality": quality,
    }


def served_quality(dev, trace, results, samples=1 << 16):
    """Quality of every served run's final population, computed on the
    device: IGD against the run's unit reference directions (points of the
    synthetic law's optimal front, the unit sphere), and the normalized
    hypervolume of the paper's box for that front (f_min = 0, f_max = 1:
    ideal 0, reference point 1.01), from `samples` sample points. Means per
    objective count."""
    import numpy as np
    import torch

    from paper_2504_06067_amd import nsga3

    by_m = {}
    t0 = time.perf_counter()
    for q in trace:
        F = torch.from_numpy(np.ascontiguousarray(results[q["rid"]]["F"])).to(dev)
        Z = np.asarray(q["Z"], np.float64)
        R = torch.from_numpy((Z / np.linalg.norm(Z, axis=1, keepdims=True)).astype(np.float32)).to(dev)
        m = F.shape[1]
        igd = nsga3.igd(F, R)
        hv = nsga3.hv_count(F, [0.0] * m, [1.01] * m, samples, q["rid"])
        torch.cuda.synchronize(dev)
        e = by_m.setdefault(m, {"runs": 0, "igd": [], "hv": []})
        e["runs"] += 1
        e["igd"].append(float(igd.cpu()[0]))
        e["hv"].append(int(hv.cpu()[0]) / samples)
    out = {"front": "unit sphere (the synthetic law's optimum); HV box ideal 0, ref 1.01",
           "hv_samples": samples, "seconds": time.perf_counter() - t0, "by_m": {}}
    for m, e in sorted(by_m.items()):
        out["by_m"][str(m)] = {"runs": e["runs"], "igd_mean": float(np.mean(e["igd"])),
                               "igd_max": float(np.max(e["igd"])),
                               "hv_norm_mean": float(np.mean(e["hv"]))}
    return out


# Per-generation runtime of TensorNSGA-III in the paper's Table I (V100 + EPYC
# 9654, DTLZ3, m = 6, d = 500, whole generation), seconds, by population n.
# Context only: another machine, another problem.
PAPER_TABLE1_S = {50: 1.120e-3, 100: 1.135e-3, 200: 1.121e-3, 400: 1.243e-3, 800: 1.493e-3,
                  1600: 2.063e-3, 3200: 4.886e-3, 6400: 1.575e-2, 12800: 5.966e-2}


def bench_generation_loop(args, dev):
    """The whole generation on the device at the paper's Table I shapes:
    m = 6 objectives, d = 500 decision variables, population n from 50 to
    12800 (2n merged), Das-Dennis references with the count nearest n. One
    generation is the offspring step (random mating, SBX, polynomial
    mutation, synthetic objective map: nsga3_evolve_batched) and the
    selection of n from the 2n merged points (nsga3_select), both enqueued
    on one stream with the population resident; the first generation starts
    from a uniform random population. Per-generation time = HIP-event time
    of `reps` consecutive generations / reps, after 3 untimed ones."""
    import math

    import numpy as np
    import torch

    from paper_2504_06067_amd import nsga3, workloads

    m, d = 6, 500
    out = []
    for n in sorted(PAPER_TABLE1_S):
        p = min(range(1, 30), key=lambda q: (abs(math.comb(q + m - 1, m - 1) - n), q))
        Z = torch.from_numpy(workloads.das_dennis(m, p)).to(dev)
        H = Z.shape[0]
        A = torch.from_numpy(np.random.default_rng(n).standard_normal((m, d - 1))
                             .astype(np.float32)).to(dev)
        M = 2 * n
        X = [torch.empty(M * d, dtype=torch.float32, device=dev) for _ in range(2)]
        F = [torch.empty(M * m, dtype=torch.float32, device=dev) for _ in range(2)]
        sel = torch.empty(n, dtype=torch.int32, device=dev)
        ws = nsga3.Workspace(dev)
        evo_ws = nsga3.Workspace(dev)
        seed = 1000 + n
        nsga3.evolve(nsga3.EVOLVE_INIT, n, d, m, A, seed, 0, X[0], F[0], ws=evo_ws)
        state = {"cur": 0, "g": 0, "has_sel": False}
        stream = torch.cuda.current_stream(dev)

        def generation(ev=None):
            cur, g = state["cur"], state["g"]
            nsga3.evolve(nsga3.EVOLVE_GENERATION, n, d, m, A, seed, g + 1, X[1 - cur], F[1 - cur],
                         X_old=X[cur], F_old=F[cur], sel=sel if state["has_sel"] else None,
                         ws=evo_ws)
            if ev is not None:
                ev.record(stream)
            nsga3.select(F[1 - cur].view(M, m), Z, n, seed ^ (g + 1), ws=ws, out=sel)
            state.update(cur=1 - cur, g=g + 1, has_sel=True)

        for _ in range(3):
            generation()
        torch.cuda.synchronize(dev)
        reps = 20 if n <= 3200 else 10
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        mids = [torch.cuda.Event(enable_timing=True) for _ in range(reps)]
        ends = [torch.cuda.Event(enable_timing=True) for _ in range(reps)]
        starts = [torch.cuda.Event(enable_timing=True) for _ in range(reps)]
        t0.record(stream)
        for i in range(reps):
            starts[i].record(stream)
            generation(mids[i])
            ends[i].record(stream)
        t1.record(stream)
        torch.cuda.synchronize(dev)
        if ws.status() != nsga3.OK:
            raise RuntimeError(f"status not OK in the generation loop at n={n}")
        per = t0.elapsed_time(t1) / reps
        evo = float(np.mean([a.elapsed_time(b) for a, b in zip(starts, mids)]))
        sel_ms = float(np.mean([a.elapsed_time(b) for a, b in zip(mids, ends)]))
        out.append({"n": n, "merged": M, "m": m, "d": d, "p": p, "H": H,
                    "ms_per_generation": per, "evolve_ms": evo, "select_ms": sel_ms,
                    "paper_tensornsga3_ms": PAPER_TABLE1_S[n] * 1e3})
        print(f"generation loop n={n}: {per:.3f} ms/generation", file=sys.stderr, flush=True)
    return {"workload": "whole generation (evolve + select) at m=6, d=500, synthetic objective "
                        "map standing in for DTLZ3; paper figures are V100 + EPYC 9654, context only",
            "points": out}


# Per-generation runtime of TensorNSGA-III in the paper's Table II (V100 + EPYC
# 9654, DTLZ3, 2n = 1600, d = 1000, whole generation), seconds, by m.
# Context only: another machine, another problem, and here selection only.
PAPER_TABLE2_S = {4: 4.334e-3, 8: 4.624e-3, 16: 5.083e-3, 32: 6.514e-3, 64: 8.103e-3,
                  128: 1.016e-2, 256: 2.348e-2, 512: 3.199e-2}


def bench_objective_scaling(args, dev, reps=20):
    """Selection at the paper's objective-scaling shapes: 2N = 1600 merged
    points (radius law of the large workload), m from 4 to 512, Das-Dennis
    references with the count nearest N = 800. p50 of `reps` selections (HIP
    events), with the dominance, normalization and association kernels'
    average times."""
    import math

    import numpy as np
    import torch

    from paper_2504_06067_amd import nsga3, workloads

    out = []
    M, N = 1600, 800
    for m in sorted(PAPER_TABLE2_S):
        p = min(range(1, 40), key=lambda q: (abs(math.comb(q + m - 1, m - 1) - N), q))
        inst = dict(F=workloads.objectives(np.random.default_rng(m), M, m, "exp"),
                    Z=workloads.das_dennis(m, p), M=M, m=m, N=N, seed=m)
        inst["H"] = len(inst["Z"])
        r = plain_steps(inst, dev, reps, 3,
                        profile="dominance,peel,norm_fused,norm_reduce,norm_extreme,norm_solve,"
                                "associate,niche_plan")
        t = r["step_ms"]
        k = {n: round(v["avg_us"], 1) for n, v in r["kernels"].items() if v["launches"]}
        out.append({"m": m, "merged": M, "p": p, "H": inst["H"],
                    "select_ms_p50": float(np.percentile(t, 50)),
                    "select_ms_p99": float(np.percentile(t, 99)),
                    "kernels_avg_us": k,
                    "paper_tensornsga3_generation_ms": PAPER_TABLE2_S[m] * 1e3})
        print(f"objective scaling m={m}: {out[-1]['select_ms_p50']:.3f} ms", file=sys.stderr,
              flush=True)
    return {"workload": "selection of N=800 from 2N=1600 at m = 4..512 (synthetic radius law "
                        "standing in for DTLZ3); paper figures are whole generations on a V100, "
                        "context only",
            "points": out}


def plain_steps(inst, dev, steps, warmup, profile=None):
    """Times `steps` plain selections of one instance (inputs resident in HBM):
    wall time over the whole loop, per-step HIP events on the stream, and the
    summed HIP-event time of the kernels named in `profile`."""
    import numpy as np
    import torch

    from paper_2504_06067_amd import nsga3

    F = torch.from_numpy(inst["F"]).to(dev)
    Z = torch.from_numpy(inst["Z"]).to(dev)
    ws = nsga3.Workspace(dev)
    out = torch.empty(inst["N"], dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)
    for _ in range(warmup):
        nsga3.select(F, Z, inst["N"], inst["seed"], ws=ws, out=out)
    torch.cuda.synchronize(dev)
    if ws.status() != nsga3.OK:
        raise RuntimeError("device status not OK after warm-up")
    if profile:
        nsga3.profile_enable(profile)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    stops = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for i in range(steps):
        starts[i].record(stream)
        nsga3.select(F, Z, inst["N"], inst["seed"], ws=ws, out=out)
        stops[i].record(stream)
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t0
    kern = {}
    if profile:
        for name in profile.split(","):
            ms, n, dropped = nsga3.profile_read(name)
            kern[name] = {"avg_us": ms / max(n, 1) * 1e3, "launches": n, "dropped": dropped}
        nsga3.profile_enable(None)
    if ws.status() != nsga3.OK:
        raise RuntimeError("device status not OK after the timed region")
    step_ms = np.array([a.elapsed_time(b) for a, b in zip(starts, stops)])
    gpu_out = nsga3.select(F, Z, inst["N"], inst["seed"], ws=ws, intermediates=True)
    torch.cuda.synchronize(dev)
    return dict(wall=wall, step_ms=step_ms, kernels=kern, gpu_out=gpu_out)


KERNELS = ("header,prep,place_scatter,place_gather,dominance,peel,norm_fused,norm_reduce,norm_extreme,associate,assoc_final,"
           "niche_plan,niche_scatter,niche_pick,compact")


PLACE_BUCKETS = 1024  # first-objective buckets of the library's point placement


def dominance_work(F):
    """Work of one dominance launch on objective set F [M][m], from a host
    replica of the library's placement (the same float32 bucket function,
    so the same tile kinds): an ordered tile (column block wholly in lower
    buckets) costs m - 1 compares and one shift per column point, a full
    tile 2m compares, one shift and two lane writes. Counts are per launch,
    in lane operations (64 per wave instruction)."""
    import numpy as np

    F = np.asarray(F, np.float32)
    M, m = F.shape
    f1 = F[:, 0]
    # the library's bucket range: a strided sample of 256 points
    sample = f1[(np.arange(256, dtype=np.int64) * M) >> 8]
    lo, hi = sample.min(), sample.max()
    span = np.float32(hi - lo)
    scale = np.float32(PLACE_BUCKETS) / span if (span > 0 and np.isfinite(span)) else np.float32(0)
    t = (f1 - lo) * scale
    b = np.where(t >= PLACE_BUCKETS, PLACE_BUCKETS - 1, np.where(t > 0, np.floor(t), 0)).astype(np.int64)
    start = np.concatenate([[0], np.cumsum(np.bincount(b, minlength=PLACE_BUCKETS))])
    W = (M + 63) // 64
    bs = np.sort(b)
    first_bucket = bs[64 * np.arange(W)]
    row_ord = start[first_bucket] >> 6               # ordered tiles per row block
    last_bucket = bs[np.minimum(64 * np.arange(W) + 63, M - 1)]
    col_end = (start[last_bucket + 1] + 63) >> 6     # the peel's column bound
    ordered = int(row_ord.sum())
    full = W * (W + 1) // 2 - ordered                # includes the W diagonal tiles
    lanes = 64 * 64                                  # column points x lanes per tile
    compares = lanes * (ordered * (m - 1) + full * 2 * m)
    valu = lanes * (ordered * m + full * (2 * m + 3))
    # words written: one per row-block lane per tile, and the reverse word
    # of full off-diagonal tiles; the objective copy read once
    bytes_ = (ordered + full + (full - W)) * 64 * 8 + M * m * 4
    return {"tiles_ordered": ordered, "tiles_full": full, "compare_lane_ops": compares,
            "valu_lane_ops": valu, "pairs": M * (M - 1) // 2, "algorithmic_bytes": bytes_,
            "column_bytes": int(col_end.sum()) * 64 * 8}


def dominance_roofline(F, avg_s):
    """VALU issue rate of the dominance kernel against the issue peak, with
    the compares alone and the classic 2m compares per unordered pair beside
    it (what the formulation without placement executes)."""
    w = dominance_work(F)
    m = len(F[0])
    # from six objectives a wave leaves a compare chain early once no lane
    # is left, so the count (every compare) bounds what executes
    unit = ("T VALU lane-ops/s (executed: compares, shifts, lane writes)" if m < 6 else
            "T VALU lane-ops/s (every compare of the chains counted; the kernel skips the "
            "rest of a chain once no lane is left, so fewer execute)")
    out = {"achieved": w["valu_lane_ops"] / avg_s / 1e12, "peak": VALU_PEAK_OPS / 1e12,
           "unit": unit,
           "frac": w["valu_lane_ops"] / avg_s / VALU_PEAK_OPS,
           "compare_frac": w["compare_lane_ops"] / avg_s / VALU_PEAK_OPS,
           "classic_2m_per_pair_frac": w["pairs"] * 2 * m / avg_s / VALU_PEAK_OPS,
           "tiles_ordered": w["tiles_ordered"], "tiles_full": w["tiles_full"],
           "algorithmic_bytes": w["algorithmic_bytes"]}
    return out


def kernel_rooflines(inst, dev, reps):
    """Per-kernel average times of a separate profiled pass (not the timed
    region), with the association against the VALU issue peak and the peel's
    matrix reads against HBM."""
    import numpy as np

    r = plain_steps(inst, dev, reps, 3, profile=KERNELS)
    k = r["kernels"]
    rank = r["gpu_out"]["rank"].cpu().numpy()
    from paper_2504_06067_amd import nsga3
    l = int(rank[rank != nsga3.UNRANKED].max())
    st = int(np.sum(rank <= l))
    M, m, H = inst["M"], inst["m"], inst["H"]
    W = (M + 63) // 64
    pairs = st * H
    a_s = k["associate"]["avg_us"] / 1e6
    p_s = k["peel"]["avg_us"] / 1e6
    # the words the peel reads: each column below its placement bound
    col_bytes = dominance_work(inst["F"])["column_bytes"]
    return {
        "kernels_avg_us": {n: round(v["avg_us"], 2) for n, v in k.items()},
        "sum_kernels_us": round(sum(v["avg_us"] for v in k.values()), 1),
        # executed per pair: 3m for the residual distance, and per group of
        # eight references four min operations and four for the compare with
        # the running best (about one per pair); the residual form priced
        # reference by reference (a compare and two selects) is 3m + 3
        "associate": {"bound": "alu", "pairs": pairs,
                      "lane_ops_per_pair": 3 * m + 1,
                      "achieved": pairs * (3 * m + 1) / a_s / 1e12,
                      "peak": VALU_PEAK_OPS / 1e12, "unit": "T lane-ops/s",
                      "frac": pairs * (3 * m + 1) / a_s / VALU_PEAK_OPS,
                      "residual_form_3m_plus_3_frac": pairs * (3 * m + 3) / a_s / VALU_PEAK_OPS,
                      "flops_2m_per_pair_tflops": pairs * 2 * m / a_s / 1e12},
        "peel": {"bound": "latency", "fronts": l + 1, "column_bytes": col_bytes,
                 "mask_bytes": W * W * 64 * 8,
                 "achieved_one_column_pass_gbs": col_bytes / p_s / 1e9, "peak_gbs": 8000.0,
                 "frac_one_column_pass": col_bytes / p_s / 8e12},
    }


def latency_leg(name, dev, seed, reps, warmup):
    """p50/p99 step latency (HIP events) and throughput of one plain workload."""
    import numpy as np

    from paper_2504_06067_amd import workloads

    inst = workloads.plain_instance(name, seed)
    r = plain_steps(inst, dev, reps, warmup, profile="dominance,select_tiny")
    t = r["step_ms"]
    dom = r["kernels"]["dominance"]
    tiny = r["kernels"]["select_tiny"]
    out = {
        "workload": f"plain selection, 2N={inst['M']}, m={inst['m']}, H={inst['H']}, N={inst['N']}",
        "reps": reps,
        "latency_ms": {"p50": float(np.percentile(t, 50)), "p99": float(np.percentile(t, 99)),
                       "mean": float(t.mean())},
        "value": inst["M"] * reps / r["wall"],
        "value_at_p50": inst["M"] / (float(np.percentile(t, 50)) / 1e3),
        "unit": "merged solutions/s",
    }
    if dom["launches"]:
        out["dominance"] = dominance_roofline(inst["F"], dom["avg_us"] / 1e6)
        out["dominance_avg_us"] = dom["avg_us"]
    if tiny["launches"]:
        # the one-workgroup path: the whole selection in one launch
        out["path"] = "one workgroup (one launch)"
        out["select_tiny_avg_us"] = tiny["avg_us"]
    return out, inst, r["gpu_out"]


def bench_niche_ab(dev, legs, reps=30):
    """The niche stage alone on each workload's own (rank, front_info, pi,
    dist) from the GPU: the closed form (nsga3_niche) against the paper's
    cache-tensor loop (nsga3_niche_cache_tensor); per-call p50 and the
    kernel times of each, and whether the selections are identical."""
    import numpy as np
    import torch

    from paper_2504_06067_amd import nsga3

    out = {}
    stream = torch.cuda.current_stream(dev)
    for name, (inst, g) in legs.items():
        rank, pi, dist = g["rank"], g["pi"], g["dist"]
        rk = rank.cpu().numpy()
        l = int(rk[rk != nsga3.UNRANKED].max())
        S = int(np.sum(rk < l))
        fi = torch.tensor([l, S, inst["N"] - S, l + 1], dtype=torch.int32, device=dev)
        res = {"l": l, "S": S, "K": inst["N"] - S, "H": inst["H"]}
        sels = {}
        for label, ct, kern in (("closed_form", False, "niche_scatter,niche_plan,niche_pick,compact"),
                                ("cache_tensor", True, "niche_scatter,ct_offsets,ct_order,ct_loop,compact")):
            ws = nsga3.Workspace(dev)
            for _ in range(3):
                nsga3.niche(rank, fi, pi, dist, inst["H"], inst["N"], inst["seed"], ws=ws,
                            cache_tensor=ct)
            torch.cuda.synchronize(dev)
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(reps)]
            nsga3.profile_enable(kern)
            for a, b in ev:
                a.record(stream)
                sel = nsga3.niche(rank, fi, pi, dist, inst["H"], inst["N"], inst["seed"], ws=ws,
                                  cache_tensor=ct)
                b.record(stream)
            torch.cuda.synchronize(dev)
            kt = {}
            for k in kern.split(","):
                ms, n, _ = nsga3.profile_read(k)
                kt[k] = round(ms / max(n, 1) * 1e3, 2)
            nsga3.profile_enable(None)
            ms = np.array([a.elapsed_time(b) for a, b in ev])
            res[label] = {"p50_us": float(np.percentile(ms, 50)) * 1e3, "kernels_avg_us": kt,
                          "status": ws.status()}
            sels[label] = sel.cpu().numpy()
        res["identical"] = bool(np.array_equal(sels["closed_form"], sels["cache_tensor"]))
        res["speedup_closed_form"] = res["cache_tensor"]["p50_us"] / res["closed_form"]["p50_us"]
        out[name] = res
        print(f"niche A/B {name}: closed form {res['closed_form']['p50_us']:.1f} us, cache tensor "
              f"{res['cache_tensor']['p50_us']:.1f} us, identical {res['identical']}",
              file=sys.stderr, flush=True)
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the selection path is single-GPU "
              "(multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2504_06067_amd import workloads

    dev = torch.device("cuda:0")
    if args.only_batched:
        print(json.dumps({"batched": bench_batched(args, dev)}), flush=True)
        return
    if args.only_served:
        print(json.dumps({"served": bench_served(args, dev)}), flush=True)
        return
    inst = workloads.plain_instance(args.workload, args.seed)
    M, m, H, N = inst["M"], inst["m"], inst["H"], inst["N"]
    if args.calib_copy_mb:
        n = args.calib_copy_mb << 20
        src = torch.ones(n, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize(dev)
        del src, dst

    dominant = "dominance"
    r = plain_steps(inst, dev, args.steps, args.warmup, profile=dominant)
    print(f"timed {args.steps} steps of {args.workload}", file=sys.stderr, flush=True)
    wall, step_ms = r["wall"], r["step_ms"]
    main_out = r["gpu_out"]
    from paper_2504_06067_amd import profiling
    rec = profiling.read_traffic(os.path.join(ROOT, "profiles", f"k_dominance_{args.workload}_traffic.json"))
    traffic = rec["traffic_bytes"] if rec else None
    dom_avg_s = r["kernels"][dominant]["avg_us"] / 1e6
    dom_rl = dominance_roofline(inst["F"], dom_avg_s)

    res = {
        "metric": METRIC,
        "value": M * args.steps / wall,
        "unit": "merged solutions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"plain selection, 2N={M}, m={m}, H={H} (Das-Dennis p={workloads.PLAIN[args.workload]['p']}), "
                        f"N={N}, law={workloads.PLAIN[args.workload]['law']}",
            "global_batch": M,
            "seq_len": None,
            "parallelism": "single GPU",
        },
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)), "p99": float(np.percentile(step_ms, 99)),
                       "mean": float(step_ms.mean())},
        "roofline": {
            "kernel": "k_dominance",
            "bound": "alu",
            "achieved": dom_rl["achieved"],
            "peak": dom_rl["peak"],
            "unit": dom_rl["unit"],
            "frac": dom_rl["frac"],
            "compare_frac": dom_rl["compare_frac"],
            "classic_2m_per_pair_frac": dom_rl["classic_2m_per_pair_frac"],
            "tiles_ordered": dom_rl["tiles_ordered"],
            "tiles_full": dom_rl["tiles_full"],
            "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by "
                            "a plain copy of known size)",
            "algorithmic_bytes": dom_rl["algorithmic_bytes"],
            "avg_kernel_ms": dom_avg_s * 1e3,
            "launches_timed": r["kernels"][dominant]["launches"],
        },
    }
    if not args.no_kernels:
        res["kernels"] = kernel_rooflines(inst, dev, 20)
    legs = {}
    if not args.no_configs:
        small, small_inst, small_out = latency_leg("small", dev, args.seed, args.small_reps, 50)
        many, many_inst, many_out = latency_leg("many_objective", dev, args.seed, args.many_reps, 3)
        res["small"] = small
        res["many_objective"] = many
        legs = {"small": (small_inst, small_out), "many_objective": (many_inst, many_out)}
        print("timed the small and many-objective workloads", file=sys.stderr, flush=True)
    if not args.no_niche_ab:
        ab_legs = {args.workload: (inst, main_out)}
        ab_legs.update({k: v for k, v in legs.items() if k != "small"})
        res["niche_ab"] = bench_niche_ab(dev, ab_legs)
    if not args.no_generations:
        res["generation_loop"] = bench_generation_loop(args, dev)
    if not args.no_objective_scaling:
        res["objective_scaling"] = bench_objective_scaling(args, dev)
    if not args.no_batched:
        res["batched"] = bench_batched(args, dev)
        print("timed the batched workload", file=sys.stderr, flush=True)
    if not args.no_served:
        res["served"] = bench_served(args, dev)
        print("timed the served workload", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(inst, args.cpu_seconds)
        threads = res["cpu_baseline"]["all_cores"]["cores"]
        parity = {args.workload: parity_report(dev, main_out, inst, threads)}
        for name, (q, o) in legs.items():
            parity[name] = parity_report(dev, o, q, threads)
        res["parity"] = parity
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
