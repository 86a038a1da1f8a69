"""Python binding of libnsga3.so (argument marshalling only).

Every function takes and returns torch tensors on the GPU, checks dtypes and
shapes, allocates outputs and the workspace with torch, and calls the C-ABI
declared in ``include/nsga3.h`` on the current HIP stream. All arithmetic
runs in the library's HIP kernels; there is no fallback: if the library is
missing the first call raises.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnsga3.so")

OK, EINVAL, EWORKSPACE, EHIP, ENONFINITE, EINTERNAL = 0, -1, -2, -3, -4, -5
UNRANKED = 0x7FFFFFFF
MAX_BATCH = 1024
_NAMES = {0: "OK", -1: "EINVAL", -2: "EWORKSPACE", -3: "EHIP", -4: "ENONFINITE", -5: "EINTERNAL"}

_lib = None


class Nsga3Error(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {_NAMES.get(code, code)}")
        self.code = code


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libnsga3.so not built at {LIB_PATH}; run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, u64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_size_t
    L.nsga3_workspace_bytes.argtypes = [i32, i32, i32, i32]
    L.nsga3_workspace_bytes.restype = sz
    L.nsga3_nd_sort.argtypes = [P, i32, i32, i32, P, P, P, sz, P]
    L.nsga3_normalize.argtypes = [P, P, P, i32, i32, P, P, P, P, P, P, sz, P]
    L.nsga3_associate.argtypes = [P, P, P, i32, i32, P, i32, P, P, P, sz, P]
    L.nsga3_niche.argtypes = [P, P, P, P, i32, i32, i32, u64, P, P, sz, P]
    L.nsga3_niche_cache_tensor.argtypes = [P, P, P, P, i32, i32, i32, u64, P, P, sz, P]
    L.nsga3_select.argtypes = [P, i32, i32, P, i32, i32, u64, P, P, P, P, P, sz, P]
    L.nsga3_select_noalloc.argtypes = [P, i32, i32, P, i32, i32, u64, P, P, P, P, P, P]
    L.nsga3_read_status.argtypes = [P, P, P]
    L.nsga3_batched_workspace_bytes.argtypes = [P, i32]
    L.nsga3_batched_workspace_bytes.restype = sz
    L.nsga3_select_batched.argtypes = [P, i32, P, sz, P]
    L.nsga3_read_status_batched.argtypes = [P, i32, P, P, P]
    L.nsga3_instance_workspace_bytes.argtypes = [i32, i32, i32, i32]
    L.nsga3_instance_workspace_bytes.restype = sz
    L.nsga3_evolve_workspace_bytes.argtypes = [i32]
    L.nsga3_evolve_workspace_bytes.restype = sz
    L.nsga3_evolve_batched.argtypes = [P, i32, P, sz, P]
    L.nsga3_igd_workspace_bytes.argtypes = [i32]
    L.nsga3_igd_workspace_bytes.restype = sz
    L.nsga3_igd.argtypes = [P, i32, i32, P, i32, P, P, sz, P]
    L.nsga3_hv_count.argtypes = [P, i32, i32, P, P, ctypes.c_int64, u64, P, P]
    L.nsga3_version.restype = ctypes.c_char_p
    L.nsga3_profile_enable.argtypes = [ctypes.c_char_p]
    L.nsga3_profile_read.argtypes = [ctypes.c_char_p, P, P, P]
    for f in ("nsga3_nd_sort", "nsga3_normalize", "nsga3_associate", "nsga3_niche",
              "nsga3_niche_cache_tensor",
              "nsga3_select", "nsga3_select_noalloc", "nsga3_read_status", "nsga3_profile_enable", "nsga3_profile_read",
              "nsga3_select_batched", "nsga3_read_status_batched", "nsga3_evolve_batched",
              "nsga3_igd", "nsga3_hv_count"):
        getattr(L, f).restype = i32
    _lib = L
    return L


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check(rc, what):
    if rc != OK:
        raise Nsga3Error(rc, what)


def status_from_bits(bits):
    """Public status code of a raw status word read from a workspace region
    (non-finite input first, then an invalid reference row, then internal)."""
    if bits & 1:
        return ENONFINITE
    if bits & 2:
        return EINVAL
    if bits & 4:
        return EINTERNAL
    return OK


def workspace_bytes(M, m, H, N):
    return int(lib().nsga3_workspace_bytes(int(M), int(m), int(H), int(N)))


class Workspace:
    """A reusable device workspace, grown on demand (allocation happens here,
    never inside a library call)."""

    def __init__(self, device="cuda"):
        self.device = torch.device(device)
        self.buf = None

    def get(self, nbytes):
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=self.device)
        return self.buf

    def status(self):
        st = ctypes.c_int32(0)
        _check(lib().nsga3_read_status(_ptr(self.buf), _stream(self.device), ctypes.byref(st)),
               "nsga3_read_status")
        return st.value


def _f32(t, name, dims):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32 and t.dim() == dims):
        raise ValueError(f"{name} must be a {dims}-D float32 CUDA tensor")
    return t.contiguous()


def _i32(t, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.int32):
        raise ValueError(f"{name} must be an int32 CUDA tensor")
    return t.contiguous()


def nd_sort(F, n_stop=0, ws=None):
    """(rank int32[M], front_info int32[4]) of the objective matrix F [M][m]."""
    F = _f32(F, "F", 2)
    M, m = F.shape
    ws = ws or Workspace(F.device)
    buf = ws.get(workspace_bytes(M, m, 1, M))
    rank = torch.empty(M, dtype=torch.int32, device=F.device)
    fi = torch.empty(4, dtype=torch.int32, device=F.device)
    _check(lib().nsga3_nd_sort(_ptr(F), M, m, int(n_stop), _ptr(rank), _ptr(fi), _ptr(buf),
                               buf.numel(), _stream(F.device)), "nsga3_nd_sort")
    return rank, fi


def normalize(F, rank, front_info, ws=None):
    """dict(Fn, ideal, intercept, extreme, degenerate) over S_t."""
    F = _f32(F, "F", 2)
    rank, front_info = _i32(rank, "rank"), _i32(front_info, "front_info")
    M, m = F.shape
    ws = ws or Workspace(F.device)
    buf = ws.get(workspace_bytes(M, m, 1, M))
    dev = F.device
    Fn = torch.zeros((M, m), dtype=torch.float32, device=dev)
    ideal = torch.empty(m, dtype=torch.float32, device=dev)
    icpt = torch.empty(m, dtype=torch.float64, device=dev)
    ext = torch.empty(m, dtype=torch.int32, device=dev)
    deg = torch.empty(1, dtype=torch.int32, device=dev)
    _check(lib().nsga3_normalize(_ptr(F), _ptr(rank), _ptr(front_info), M, m, _ptr(Fn), _ptr(ideal),
                                 _ptr(icpt), _ptr(ext), _ptr(deg), _ptr(buf), buf.numel(),
                                 _stream(dev)), "nsga3_normalize")
    return dict(Fn=Fn, ideal=ideal, intercept=icpt, extreme=ext, degenerate=deg)


def associate(Fn, rank, front_info, Z, ws=None):
    """(pi int32[M], dist float32[M]); -1 outside S_t."""
    Fn, Z = _f32(Fn, "Fn", 2), _f32(Z, "Z", 2)
    rank, front_info = _i32(rank, "rank"), _i32(front_info, "front_info")
    M, m = Fn.shape
    H = Z.shape[0]
    if Z.shape[1] != m:
        raise ValueError("Z must have m columns")
    ws = ws or Workspace(Fn.device)
    buf = ws.get(workspace_bytes(M, m, H, M))
    pi = torch.empty(M, dtype=torch.int32, device=Fn.device)
    dist = torch.empty(M, dtype=torch.float32, device=Fn.device)
    _check(lib().nsga3_associate(_ptr(Fn), _ptr(rank), _ptr(front_info), M, m, _ptr(Z), H, _ptr(pi),
                                 _ptr(dist), _ptr(buf), buf.numel(), _stream(Fn.device)),
           "nsga3_associate")
    return pi, dist


def niche(rank, front_info, pi, dist, H, N, seed, ws=None, cache_tensor=False):
    """Ascending selected indices int32[N]. cache_tensor=True runs the paper's
    cache-tensor loop (nsga3_niche_cache_tensor) instead of the closed form."""
    rank, front_info, pi = _i32(rank, "rank"), _i32(front_info, "front_info"), _i32(pi, "pi")
    if not (dist.is_cuda and dist.dtype == torch.float32):
        raise ValueError("dist must be a float32 CUDA tensor")
    dist = dist.contiguous()
    M = rank.shape[0]
    ws = ws or Workspace(rank.device)
    buf = ws.get(workspace_bytes(M, 2, H, N))
    sel = torch.empty(int(N), dtype=torch.int32, device=rank.device)
    fn = lib().nsga3_niche_cache_tensor if cache_tensor else lib().nsga3_niche
    _check(fn(_ptr(rank), _ptr(front_info), _ptr(pi), _ptr(dist), M, int(H), int(N),
              int(seed) & (2**64 - 1), _ptr(sel), _ptr(buf), buf.numel(), _stream(rank.device)),
           "nsga3_niche_cache_tensor" if cache_tensor else "nsga3_niche")
    return sel


def select(F, Z, N, seed, ws=None, out=None, intermediates=False):
    """The whole selection. Returns the ascending selected indices, or with
    intermediates=True a dict(selected, rank, pi, dist)."""
    F, Z = _f32(F, "F", 2), _f32(Z, "Z", 2)
    M, m = F.shape
    H = Z.shape[0]
    if Z.shape[1] != m:
        raise ValueError("Z must have m columns")
    dev = F.device
    ws = ws or Workspace(dev)
    buf = ws.get(workspace_bytes(M, m, H, N))
    sel = out if out is not None else torch.empty(int(N), dtype=torch.int32, device=dev)
    rank = pi = dist = None
    if intermediates:
        rank = torch.empty(M, dtype=torch.int32, device=dev)
        pi = torch.empty(M, dtype=torch.int32, device=dev)
        dist = torch.empty(M, dtype=torch.float32, device=dev)
    _check(lib().nsga3_select(_ptr(F), M, m, _ptr(Z), H, int(N), int(seed) & (2**64 - 1), _ptr(sel),
                              _ptr(rank), _ptr(pi), _ptr(dist), _ptr(buf), buf.numel(),
                              _stream(dev)), "nsga3_select")
    if intermediates:
        return dict(selected=sel, rank=rank, pi=pi, dist=dist)
    return sel


def igd(F, R):
    """IGD of the population F [n][m] against front points R [nr][m]
    (float32 CUDA tensors): a float64 CUDA tensor of one element."""
    F, R = _f32(F, "F", 2), _f32(R, "R", 2)
    n, m = F.shape
    nr = R.shape[0]
    if R.shape[1] != m:
        raise ValueError("R must have m columns")
    ws = torch.empty(max(int(lib().nsga3_igd_workspace_bytes(nr)), 256), dtype=torch.uint8,
                     device=F.device)
    out = torch.empty(1, dtype=torch.float64, device=F.device)
    _check(lib().nsga3_igd(_ptr(F), n, m, _ptr(R), nr, _ptr(out), _ptr(ws), ws.numel(),
                           _stream(F.device)), "nsga3_igd")
    return out


def hv_count(F, ideal, ref, samples, seed):
    """Number of the `samples` sample points of the box [ideal, ref] that the
    population F [n][m] weakly dominates (an int64 CUDA tensor of one
    element); count / samples is the normalized hypervolume."""
    F = _f32(F, "F", 2)
    n, m = F.shape
    lo = (ctypes.c_float * m)(*[float(v) for v in ideal])
    hi = (ctypes.c_float * m)(*[float(v) for v in ref])
    out = torch.empty(1, dtype=torch.int64, device=F.device)
    _check(lib().nsga3_hv_count(_ptr(F), n, m, lo, hi, int(samples), int(seed) & (2**64 - 1),
                                _ptr(out), _stream(F.device)), "nsga3_hv_count")
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20


def select_noalloc(F, Z, N, seed, intermediates=False):
    """The whole selection on the library's own per-GPU scratch (no workspace
    argument; calls on one GPU must not overlap). Returns (selected, status)
    or, with intermediates=True, (dict(selected, rank, pi, dist), status);
    status is an int32[1] CUDA tensor that receives the call's status code."""
    F, Z = _f32(F, "F", 2), _f32(Z, "Z", 2)
    M, m = F.shape
    H = Z.shape[0]
    if Z.shape[1] != m:
        raise ValueError("Z must have m columns")
    dev = F.device
    sel = torch.empty(int(N), dtype=torch.int32, device=dev)
    st = torch.empty(1, dtype=torch.int32, device=dev)
    rank = pi = dist = None
    if intermediates:
        rank = torch.empty(M, dtype=torch.int32, device=dev)
        pi = torch.empty(M, dtype=torch.int32, device=dev)
        dist = torch.empty(M, dtype=torch.float32, device=dev)
    _check(lib().nsga3_select_noalloc(_ptr(F), M, m, _ptr(Z), H, int(N), int(seed) & (2**64 - 1),
                                      _ptr(sel), _ptr(rank), _ptr(pi), _ptr(dist), _ptr(st),
                                      _stream(dev)), "nsga3_select_noalloc")
    if intermediates:
        return dict(selected=sel, rank=rank, pi=pi, dist=dist), st
    return sel, st


class Instance(ctypes.Structure):
    """``nsga3_instance`` of the C header."""
    _fields_ = [("F", ctypes.c_void_p), ("Z", ctypes.c_void_p), ("selected", ctypes.c_void_p),
                ("rank", ctypes.c_void_p), ("pi", ctypes.c_void_p), ("dist", ctypes.c_void_p),
                ("M", ctypes.c_int32), ("m", ctypes.c_int32), ("H", ctypes.c_int32),
                ("N", ctypes.c_int32), ("seed", ctypes.c_uint64), ("tile", ctypes.c_int32 * 4),
                ("ws", ctypes.c_void_p), ("ws_bytes", ctypes.c_size_t)]


class Batch:
    """A batch of independent selections run by one nsga3_select_batched call.

    problems: sequence of dicts with F [M][m] and Z [H][m] (float32 CUDA), N,
    seed and optionally tile (up to 4 ints, 0 = the library's choice; when
    absent, the autotuned table's entry for the instance's shape). Outputs are
    allocated once here: ``selected[b]`` and, with intermediates=True,
    ``rank[b]``, ``pi[b]``, ``dist[b]``. ``run()`` enqueues the call on the
    current stream; it may be repeated (and captured in a graph)."""

    def __init__(self, problems, ws=None, intermediates=False):
        if not problems:
            raise ValueError("empty batch")
        self.B = len(problems)
        self.arr = (Instance * self.B)()
        self.selected, self.rank, self.pi, self.dist = [], [], [], []
        self._keep = []
        dev = None
        for b, q in enumerate(problems):
            F, Z = _f32(q["F"], "F", 2), _f32(q["Z"], "Z", 2)
            if dev is None:
                dev = F.device
            if F.device != dev or Z.device != dev:
                raise ValueError("all instances must be on one device")
            M, m = F.shape
            H = Z.shape[0]
            if Z.shape[1] != m:
                raise ValueError("Z must have m columns")
            N = int(q["N"])
            sel = torch.empty(N, dtype=torch.int32, device=dev)
            self.selected.append(sel)
            r = p_ = d = None
            if intermediates:
                r = torch.empty(M, dtype=torch.int32, device=dev)
                p_ = torch.empty(M, dtype=torch.int32, device=dev)
                d = torch.empty(M, dtype=torch.float32, device=dev)
            self.rank.append(r)
            self.pi.append(p_)
            self.dist.append(d)
            self._keep += [F, Z]
            e = self.arr[b]
            e.F, e.Z, e.selected = F.data_ptr(), Z.data_ptr(), sel.data_ptr()
            e.rank = r.data_ptr() if r is not None else None
            e.pi = p_.data_ptr() if p_ is not None else None
            e.dist = d.data_ptr() if d is not None else None
            e.M, e.m, e.H, e.N = M, m, H, N
            e.seed = int(q["seed"]) & (2**64 - 1)
            t = q.get("tile")
            if t is None:
                from . import autotune
                t = autotune.lookup(M, m, H)
            t = list(t)
            for i in range(4):
                e.tile[i] = int(t[i]) if i < len(t) else 0
        self.device = dev
        self.ws = ws or Workspace(dev)
        nbytes = int(lib().nsga3_batched_workspace_bytes(self.arr, self.B))
        if nbytes == 0:
            raise Nsga3Error(EINVAL, "nsga3_batched_workspace_bytes")
        self.buf = self.ws.get(nbytes)

    def run(self):
        _check(lib().nsga3_select_batched(self.arr, self.B, _ptr(self.buf), self.buf.numel(),
                                          _stream(self.device)), "nsga3_select_batched")
        return self.selected

    def status(self):
        """Per-instance status codes of the last run (waits for the stream)."""
        st = (ctypes.c_int32 * self.B)()
        _check(lib().nsga3_read_status_batched(self.arr, self.B, _ptr(self.buf),
                                               _stream(self.device), st),
               "nsga3_read_status_batched")
        return list(st)


EVOLVE_GENERATION, EVOLVE_POPULATION, EVOLVE_INIT = 0, 1, 2


class EvolveSlot(ctypes.Structure):
    """``nsga3_evolve_slot`` of the C header."""
    _fields_ = [("X_old", ctypes.c_void_p), ("sel", ctypes.c_void_p), ("F_old", ctypes.c_void_p),
                ("X_new", ctypes.c_void_p), ("F_new", ctypes.c_void_p), ("A", ctypes.c_void_p),
                ("N", ctypes.c_int32), ("d", ctypes.c_int32), ("m", ctypes.c_int32),
                ("generation", ctypes.c_int32), ("seed", ctypes.c_uint64), ("mode", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


def instance_workspace_bytes(M, m, H, N):
    return int(lib().nsga3_instance_workspace_bytes(int(M), int(m), int(H), int(N)))


def evolve_workspace_bytes(B):
    return int(lib().nsga3_evolve_workspace_bytes(int(B)))


def evolve_batched(slots, ws_buf, stream=None, device=None):
    """Enqueue one generation step for a ctypes array of EvolveSlot."""
    st = stream if stream is not None else _stream(device or ws_buf.device)
    _check(lib().nsga3_evolve_batched(slots, len(slots), _ptr(ws_buf), ws_buf.numel(), st),
           "nsga3_evolve_batched")


def evolve(mode, N, d, m, A, seed, generation, X_new, F_new, X_old=None, F_old=None, sel=None,
           ws=None):
    """One generation step of a single population (tensors on the GPU)."""
    slots = (EvolveSlot * 1)()
    e = slots[0]
    e.X_old, e.F_old, e.sel = (X_old.data_ptr() if X_old is not None else None,
                               F_old.data_ptr() if F_old is not None else None,
                               sel.data_ptr() if sel is not None else None)
    e.X_new, e.F_new, e.A = X_new.data_ptr(), F_new.data_ptr(), A.data_ptr()
    e.N, e.d, e.m, e.generation = int(N), int(d), int(m), int(generation)
    e.seed = int(seed) & (2**64 - 1)
    e.mode = int(mode)
    ws = ws or Workspace(X_new.device)
    buf = ws.get(evolve_workspace_bytes(1))
    evolve_batched(slots, buf, device=X_new.device)


def batched_workspace_bytes(problems):
    """Workspace bytes of a batch given (M, m, H, N) tuples (0 if rejected)."""
    arr = (Instance * len(problems))()
    for e, (M, m, H, N) in zip(arr, problems):
        e.M, e.m, e.H, e.N = M, m, H, N
    return int(lib().nsga3_batched_workspace_bytes(arr, len(problems)))


def version():
    return lib().nsga3_version().decode()


def profile_enable(names):
    """Record HIP events around launches of the named kernels ("*" = all,
    None or "" = off)."""
    _check(lib().nsga3_profile_enable(names.encode() if names else None), "nsga3_profile_enable")


def profile_read(kernel):
    """(total_ms, launches, dropped) recorded for `kernel` since the last enable."""
    tot = ctypes.c_double(0)
    n = ctypes.c_int64(0)
    dropped = ctypes.c_int32(0)
    _check(lib().nsga3_profile_read(kernel.encode(), ctypes.byref(tot), ctypes.byref(n),
                                    ctypes.byref(dropped)), "nsga3_profile_read")
    return tot.value, n.value, dropped.value
