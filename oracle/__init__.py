"""CPU oracle for NSGA-III environmental selection -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper over ``liboracle_nsga3.so`` (plain C, FP64; see
``nsga3_oracle.c`` for the paper passages each function follows). Only the
test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. The product library never loads it.
"""
import ctypes
import os

import numpy as np

from . import build as _build

UNRANKED = 0x7FFFFFFF
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.LIB):
        _build.build()
    lib = ctypes.CDLL(_build.LIB)
    P = ctypes.c_void_p
    i32 = ctypes.c_int
    u64 = ctypes.c_uint64
    lib.oracle_set_threads.argtypes = [i32]
    lib.oracle_set_threads.restype = i32
    lib.oracle_splitmix64.argtypes = [u64]
    lib.oracle_splitmix64.restype = u64
    lib.oracle_key.argtypes = [u64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32]
    lib.oracle_key.restype = u64
    lib.oracle_nd_sort.argtypes = [P, i32, i32, i32, P, P]
    lib.oracle_normalize.argtypes = [P, P, P, i32, i32, P, P, P, P, P]
    lib.oracle_associate.argtypes = [P, P, P, i32, i32, P, i32, P, P]
    lib.oracle_niche.argtypes = [P, P, P, P, i32, i32, i32, u64, P]
    lib.oracle_select.argtypes = [P, i32, i32, P, i32, i32, u64, P, P, P, P]
    for f in ("oracle_nd_sort", "oracle_normalize", "oracle_associate",
              "oracle_niche", "oracle_select"):
        getattr(lib, f).restype = i32
    _lib = lib
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"{what} failed with code {rc}")


def set_threads(n):
    """Threads for the dominance and association loops (1 = serial, the
    default). Results are identical for every count. Returns the count set."""
    return int(_load().oracle_set_threads(int(n)))


def splitmix64(x):
    return int(_load().oracle_splitmix64(ctypes.c_uint64(int(x) & (2**64 - 1))))


def key(seed, tag, j, L):
    return int(_load().oracle_key(int(seed) & (2**64 - 1), tag, j, L))


def nd_sort(F, n_stop=0):
    """Ranks (0-based, UNRANKED beyond the last selected front) and
    front_info = (l, |S|, K, fronts)."""
    F = np.ascontiguousarray(F, dtype=np.float32)
    M, m = F.shape
    rank = np.empty(M, np.int32)
    fi = np.empty(4, np.int32)
    _check(_load().oracle_nd_sort(_p(F), M, m, int(n_stop), _p(rank), _p(fi)), "oracle_nd_sort")
    return rank, fi


def normalize(F, rank, front_info):
    """Returns dict(Fn [M][m] fp64 (rows outside S_t are NaN), ideal, intercept,
    extreme, degenerate)."""
    F = np.ascontiguousarray(F, dtype=np.float32)
    rank = np.ascontiguousarray(rank, dtype=np.int32)
    fi = np.ascontiguousarray(front_info, dtype=np.int32)
    M, m = F.shape
    Fn = np.full((M, m), np.nan)
    ideal = np.empty(m)
    icpt = np.empty(m)
    ext = np.empty(m, np.int32)
    deg = np.zeros(1, np.int32)
    _check(_load().oracle_normalize(_p(F), _p(rank), _p(fi), M, m, _p(Fn), _p(ideal),
                                    _p(icpt), _p(ext), _p(deg)), "oracle_normalize")
    return dict(Fn=Fn, ideal=ideal, intercept=icpt, extreme=ext, degenerate=int(deg[0]))


def associate(Fn, rank, front_info, Z):
    """pi (int32, -1 outside S_t) and dist (fp64, -1 outside S_t)."""
    Fn = np.ascontiguousarray(Fn, dtype=np.float64)
    rank = np.ascontiguousarray(rank, dtype=np.int32)
    fi = np.ascontiguousarray(front_info, dtype=np.int32)
    Z = np.ascontiguousarray(Z, dtype=np.float32)
    M, m = Fn.shape
    H = Z.shape[0]
    pi = np.empty(M, np.int32)
    dist = np.empty(M, np.float64)
    _check(_load().oracle_associate(_p(Fn), _p(rank), _p(fi), M, m, _p(Z), H, _p(pi), _p(dist)),
           "oracle_associate")
    return pi, dist


def niche(rank, front_info, pi, dist, H, N, seed):
    """Ascending selected indices (int32[N])."""
    rank = np.ascontiguousarray(rank, dtype=np.int32)
    fi = np.ascontiguousarray(front_info, dtype=np.int32)
    pi = np.ascontiguousarray(pi, dtype=np.int32)
    dist = np.ascontiguousarray(dist, dtype=np.float64)
    M = rank.shape[0]
    sel = np.empty(N, np.int32)
    _check(_load().oracle_niche(_p(rank), _p(fi), _p(pi), _p(dist), M, int(H), int(N),
                                int(seed) & (2**64 - 1), _p(sel)), "oracle_niche")
    return sel


def select(F, Z, N, seed):
    """Whole selection. Returns dict(selected, rank, pi, dist)."""
    F = np.ascontiguousarray(F, dtype=np.float32)
    Z = np.ascontiguousarray(Z, dtype=np.float32)
    M, m = F.shape
    H = Z.shape[0]
    sel = np.empty(N, np.int32)
    rank = np.empty(M, np.int32)
    pi = np.empty(M, np.int32)
    dist = np.empty(M, np.float64)
    _check(_load().oracle_select(_p(F), M, m, _p(Z), H, int(N), int(seed) & (2**64 - 1),
                                 _p(sel), _p(rank), _p(pi), _p(dist)), "oracle_select")
    return dict(selected=sel, rank=rank, pi=pi, dist=dist)
