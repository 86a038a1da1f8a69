"""Serving of resident NSGA-III runs on one GPU, with continuous batching.

A request is a whole optimization run: a population of N decision vectors
kept resident in device memory for G generations. Each generation is the
offspring step (mating, SBX, polynomial mutation and the objective map:
``nsga3_evolve_batched``) followed by the environmental selection on the
2N merged objective vectors (``nsga3_select_batched``).

The server admits requests in arrival order as soon as they have arrived and
their memory fits in the HBM budget (a first-fit pool carved from one device
allocation). A request that does not fit waits; later requests that fit may
pass it, up to a bounded number of times, after which it holds the queue
until it is admitted.
Every tick advances all resident runs by one generation with one batched
launch sequence, so runs that arrive while others are on the GPU join the
next tick and share its launches. A run leaves after its last generation;
its memory is reused at once (the stream orders the reuse after its last
kernels).

The host runs at most `depth` ticks ahead of the GPU; completion times are
read from HIP events, so latency (arrival to result in host memory) is exact
on the GPU timeline. All random choices are functions of (request seed,
generation, individual, variable), so a run's result does not depend on what
else is resident: ``plain`` mode runs the same trace one request at a time
with the plain per-instance calls and gives bit-identical results.

No arithmetic of the method happens here: this module only plans memory,
builds descriptor arrays and enqueues library calls.
"""
import collections
import ctypes
import time

import numpy as np
import torch

from . import autotune, nsga3

ALIGN = 256
MASK64 = (1 << 64) - 1
DEFAULT_BUDGET = 64 << 30


def _sm64(x):
    z = (x + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def selection_seed(seed, g):
    """Tie-break seed of generation g of a run (a SplitMix64 hash)."""
    return _sm64((seed & MASK64) ^ _sm64((0xA5 << 56) | g))


def _up(n):
    return (int(n) + ALIGN - 1) // ALIGN * ALIGN


class Pool:
    """First-fit sub-allocator over one device allocation."""

    def __init__(self, nbytes, device):
        self.size = _up(nbytes)
        self.buf = torch.empty(self.size, dtype=torch.uint8, device=device)
        self.free = [(0, self.size)]

    def alloc(self, n):
        n = _up(n)
        for i, (o, s) in enumerate(self.free):
            if s >= n:
                if s == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (o + n, s - n)
                return o
        return None

    def release(self, off, n):
        n = _up(n)
        self.free.append((off, n))
        self.free.sort()
        merged = []
        for o, s in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + s)
            else:
                merged.append((o, s))
        self.free = merged

    def used(self):
        return self.size - sum(s for _, s in self.free)

    def view(self, off, count, dtype):
        es = torch.empty((), dtype=dtype).element_size()
        return self.buf[off:off + count * es].view(dtype)


def slot_layout(M, m, H, d, plain):
    """Byte offsets of one resident run's buffers (relative to its block)."""
    N = M // 2
    ws = nsga3.workspace_bytes(M, m, H, N) if plain else nsga3.instance_workspace_bytes(M, m, H, N)
    parts = [("ws", ws), ("X0", M * d * 4), ("X1", M * d * 4), ("F0", M * m * 4),
             ("F1", M * m * 4), ("sel", N * 4), ("Z", H * m * 4), ("A", m * (d - 1) * 4),
             ("Xo", N * d * 4), ("Fo", N * m * 4)]
    lay, o = {}, 0
    for name, n in parts:
        lay[name] = (o, n)
        o += _up(n)
    return lay, o


class Run:
    """One admitted request: its pool block and per-run state."""

    def __init__(self, req, pool, off, lay):
        self.req = req
        self.off = off
        self.lay = lay
        M, N, m, d = req["M"], req["N"], req["m"], req["d"]
        H = len(req["Z"])
        self.H = H

        def v(name, count, dtype):
            return pool.view(off + lay[name][0], count, dtype)

        self.ws = v("ws", lay["ws"][1], torch.uint8)
        self.X = [v("X0", M * d, torch.float32), v("X1", M * d, torch.float32)]
        self.F = [v("F0", M * m, torch.float32).view(M, m), v("F1", M * m, torch.float32).view(M, m)]
        self.sel = v("sel", N, torch.int32)
        self.Z = v("Z", H * m, torch.float32).view(H, m)
        self.A = v("A", m * (d - 1), torch.float32)
        self.Xo = v("Xo", N * d, torch.float32)
        self.Fo = v("Fo", N * m, torch.float32)
        self.tiles = autotune.lookup(M, m, H)
        self.cur = 0          # buffer holding the current population's generation
        self.g = 0            # generations done
        self.has_sel = False
        # inputs go through pinned staging buffers (kept alive with the run),
        # so admission never waits for the GPU
        zs = torch.from_numpy(np.ascontiguousarray(req["Z"], dtype=np.float32).reshape(-1))
        as_ = torch.from_numpy(np.ascontiguousarray(req["A"], dtype=np.float32).reshape(-1))
        if self.Z.is_cuda:
            zs, as_ = zs.pin_memory(), as_.pin_memory()
        self.staging = (zs, as_)
        self.Z.view(-1).copy_(zs, non_blocking=True)
        self.A.copy_(as_, non_blocking=True)


def _evo_slot(e, run, mode):
    req = run.req
    e.N, e.d, e.m = req["N"], req["d"], req["m"]
    e.seed = req["seed"] & MASK64
    e.mode = mode
    e.reserved = 0
    e.A = run.A.data_ptr()
    if mode == nsga3.EVOLVE_INIT:
        e.X_old = e.F_old = e.sel = None
        e.X_new, e.F_new = run.X[0].data_ptr(), run.F[0].data_ptr()
        e.generation = 0
        return
    e.X_old, e.F_old = run.X[run.cur].data_ptr(), run.F[run.cur].data_ptr()
    e.sel = run.sel.data_ptr() if run.has_sel else None
    if mode == nsga3.EVOLVE_POPULATION:
        e.X_new, e.F_new = run.Xo.data_ptr(), run.Fo.data_ptr()
        e.generation = run.g
    else:
        e.X_new, e.F_new = run.X[1 - run.cur].data_ptr(), run.F[1 - run.cur].data_ptr()
        e.generation = run.g + 1


class Lane:
    """One continuous batch on its own HIP stream (default priority)."""

    def __init__(self, device, max_active, stream=None):
        self.stream = stream if stream is not None else torch.cuda.Stream(device)
        self.handle = ctypes.c_void_p(self.stream.cuda_stream)
        self.max_active = max_active
        self.active = []
        self.newly = []
        self.inflight = collections.deque()
        self.evo_buf = torch.empty(nsga3.evolve_workspace_bytes(max_active), dtype=torch.uint8,
                                   device=device)
        self.hdr = nsga3.Workspace(device)


def admit_arrived(queue, now, try_admit, passed, max_bypass):
    """One admission pass over the queue (sorted by arrival): the arrived
    requests in order, each through try_admit(q) (True: admitted, False: does
    not fit now, None: can never fit, dropped). A request that does not fit
    is passed by later ones that fit, at most `max_bypass` times (counted in
    `passed`, rid -> admissions ahead of it); then it holds every later
    request until it is admitted, so a large request cannot starve. Removes
    the admitted and dropped requests from `queue`; returns how many
    admissions passed a waiting request."""
    i = bypasses = 0
    while i < len(queue) and queue[i]["arrival"] <= now:
        q = queue[i]
        r = try_admit(q)
        if r is None:
            del queue[i]
            continue
        if not r:
            if passed.get(q["rid"], 0) >= max_bypass:
                break
            i += 1
            continue
        held = False
        for k in range(i):
            rid = queue[k]["rid"]
            passed[rid] = passed.get(rid, 0) + 1
            held |= passed[rid] >= max_bypass
        del queue[i]
        bypasses += i > 0
        if held:
            break
    return bypasses


class Server:
    """Runs a request trace.

    mode "batched": continuous batching. Admitted runs go to a lane by size
    (2N below each of `lanes` thresholds, then the rest); each lane is one
    continuous batch on its own stream, so small runs are not paced by the
    generations of large ones while the GPU overlaps the lanes' kernels.
    mode "plain": one request at a time, plain per-instance calls, one stream."""

    def __init__(self, device="cuda:0", budget=DEFAULT_BUDGET, mode="batched",
                 max_batch=nsga3.MAX_BATCH, depth=2, lanes=(8192, 32768), max_bypass=8):
        if mode not in ("batched", "plain"):
            raise ValueError(mode)
        self.max_bypass = max_bypass
        self.device = torch.device(device)
        self.mode = mode
        self.plain = mode == "plain"
        self.depth = depth
        self.pool = Pool(budget, self.device)
        self.bounds = () if self.plain else tuple(sorted(lanes))
        cap = 1 if self.plain else max_batch
        self.lanes = [Lane(self.device, cap) for _ in range(len(self.bounds) + 1)]

    def _lane_of(self, M):
        for i, b in enumerate(self.bounds):
            if M < b:
                return self.lanes[i]
        return self.lanes[-1]

    # -- launches -------------------------------------------------------
    def _evolve(self, lane, runs, mode):
        arr = (nsga3.EvolveSlot * len(runs))()
        for e, r in zip(arr, runs):
            _evo_slot(e, r, mode)
        nsga3.evolve_batched(arr, lane.evo_buf, stream=lane.handle)

    def _select(self, lane, runs):
        stream = lane.handle
        if self.plain:
            for r in runs:
                req = r.req
                Fm = r.F[1 - r.cur]
                rc = nsga3.lib().nsga3_select(
                    ctypes.c_void_p(Fm.data_ptr()), req["M"], req["m"],
                    ctypes.c_void_p(r.Z.data_ptr()), r.H, req["N"],
                    selection_seed(req["seed"], r.g + 1), ctypes.c_void_p(r.sel.data_ptr()),
                    None, None, None, ctypes.c_void_p(r.ws.data_ptr()), r.ws.numel(), stream)
                nsga3._check(rc, "nsga3_select")
            return
        arr = (nsga3.Instance * len(runs))()
        for e, r in zip(arr, runs):
            req = r.req
            e.F, e.Z, e.selected = r.F[1 - r.cur].data_ptr(), r.Z.data_ptr(), r.sel.data_ptr()
            e.rank = e.pi = e.dist = None
            e.M, e.m, e.H, e.N = req["M"], req["m"], r.H, req["N"]
            e.seed = selection_seed(req["seed"], r.g + 1)
            e.ws, e.ws_bytes = r.ws.data_ptr(), r.ws.numel()
            for i, t in enumerate(r.tiles):
                e.tile[i] = t
        nbytes = int(nsga3.lib().nsga3_batched_workspace_bytes(arr, len(runs)))
        if nbytes == 0:
            raise nsga3.Nsga3Error(nsga3.EINVAL, "nsga3_batched_workspace_bytes")
        buf = lane.hdr.get(nbytes)
        nsga3._check(nsga3.lib().nsga3_select_batched(arr, len(runs), nsga3._ptr(buf), buf.numel(),
                                                      stream), "nsga3_select_batched")

    def _tick(self, lane, pending):
        """Enqueue one generation of every run of the lane (on its stream)."""
        if lane.newly:
            self._evolve(lane, lane.newly, nsga3.EVOLVE_INIT)
            lane.newly = []
        self._evolve(lane, lane.active, nsga3.EVOLVE_GENERATION)
        self._select(lane, lane.active)
        for r in lane.active:
            r.g += 1
            r.cur ^= 1
            r.has_sel = True
        done = [r for r in lane.active if r.g == r.req["generations"]]
        if done:
            self._evolve(lane, done, nsga3.EVOLVE_POPULATION)
            for r in done:
                hx = torch.empty(r.Xo.numel(), dtype=torch.float32, pin_memory=True)
                hf = torch.empty(r.Fo.numel(), dtype=torch.float32, pin_memory=True)
                hs = torch.empty(1, dtype=torch.int32, pin_memory=True)
                hx.copy_(r.Xo, non_blocking=True)
                hf.copy_(r.Fo, non_blocking=True)
                # status word of the run's last selection (start of its region)
                hs.copy_(r.ws[:4].view(torch.int32), non_blocking=True)
                ev = torch.cuda.Event(enable_timing=True)
                ev.record(lane.stream)
                pending.append((ev, r, hx, hf, hs))
            lane.active = [r for r in lane.active if r.g < r.req["generations"]]
        ev = torch.cuda.Event()
        ev.record(lane.stream)
        lane.inflight.append(ev)

    # -- the loop -------------------------------------------------------
    def run(self, trace, realtime=True):
        """Serve `trace` (list of request dicts with arrival times in
        seconds). Returns {rid: dict(X, F, latency_s, done_s, status)} plus a
        summary under key None."""
        dev = self.device
        torch.cuda.synchronize(dev)
        queue = collections.deque(sorted(trace, key=lambda q: (q["arrival"], q["rid"])))
        results, pending = {}, []
        passed = {}      # rid -> later requests admitted ahead of it
        bypasses = 0     # admissions that passed a waiting request
        t_ev = torch.cuda.Event(enable_timing=True)
        t_ev.record(torch.cuda.current_stream(dev))
        t0 = time.perf_counter()
        ticks = peak_active = peak_bytes = 0

        def now():
            return time.perf_counter() - t0 if realtime else float("inf")

        def collect(block):
            # results of finished runs; their memory returns to the pool only
            # now, after the run's last kernels and copies completed (lanes
            # run on different streams)
            keep = []
            for item in pending:
                ev, run, hx, hf, hs = item
                if not (block or ev.query()):
                    keep.append(item)
                    continue
                ev.synchronize()
                done = t_ev.elapsed_time(ev) / 1e3
                req = run.req
                results[req["rid"]] = dict(X=hx.numpy().reshape(req["N"], req["d"]),
                                           F=hf.numpy().reshape(req["N"], req["m"]),
                                           done_s=done, latency_s=done - req["arrival"],
                                           status=nsga3.status_from_bits(int(hs[0])))
                self.pool.release(run.off, run.nbytes)
            pending[:] = keep

        def busy():
            return any(lane.active for lane in self.lanes)

        def try_admit(q):
            # True: admitted; False: does not fit now; None: never fits
            lane = self._lane_of(q["M"])
            lay, nb = slot_layout(q["M"], q["m"], len(q["Z"]), q["d"], self.plain)
            if nb > self.pool.size:
                results[q["rid"]] = dict(status=nsga3.EWORKSPACE, latency_s=None, done_s=None)
                return None
            off = self.pool.alloc(nb) if len(lane.active) < lane.max_active else None
            if off is None:
                return False
            with torch.cuda.stream(lane.stream):
                run = Run(q, self.pool, off, lay)
            run.nbytes = nb
            lane.newly.append(run)
            lane.active.append(run)
            return True

        while queue or busy() or pending:
            bypasses += admit_arrived(queue, now(), try_admit, passed, self.max_bypass)
            n_active = sum(len(lane.active) for lane in self.lanes)
            peak_active = max(peak_active, n_active)
            peak_bytes = max(peak_bytes, self.pool.used())

            progressed = False
            for lane in self.lanes:
                while lane.inflight and lane.inflight[0].query():
                    lane.inflight.popleft()
                if lane.active and len(lane.inflight) < self.depth:
                    with torch.cuda.stream(lane.stream):
                        self._tick(lane, pending)
                    ticks += 1
                    progressed = True
            collect(False)
            if not progressed:
                if not busy() and not pending and queue:
                    wait = queue[0]["arrival"] - now()
                    if wait > 0:
                        time.sleep(min(wait, 0.002))
                else:
                    time.sleep(0.00005)
        torch.cuda.synchronize(dev)
        collect(True)
        makespan = max((r["done_s"] for r in results.values() if r.get("done_s") is not None),
                       default=0.0)
        results[None] = dict(ticks=ticks, makespan_s=makespan, peak_active=peak_active,
                             peak_pool_bytes=peak_bytes, bypasses=bypasses)
        return results
