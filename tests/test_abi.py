"""The C-ABI library loads and exports every function include/nsga3.h
declares; host-only behaviour (workspace sizing, argument validation) works
without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nsga3.h")
LIB = os.path.join(ROOT, "paper_2504_06067_amd", "libnsga3.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nsga3_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libnsga3.so is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(LIB)
    L.nsga3_workspace_bytes.restype = ctypes.c_size_t
    L.nsga3_workspace_bytes.argtypes = [ctypes.c_int32] * 4
    return L


def test_header_declares_the_stage_calls():
    names = declared_functions()
    for f in ["nsga3_nd_sort", "nsga3_normalize", "nsga3_associate", "nsga3_niche",
              "nsga3_select", "nsga3_workspace_bytes", "nsga3_read_status", "nsga3_version"]:
        assert f in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_workspace_bytes(lib):
    ws = lib.nsga3_workspace_bytes
    assert ws(1, 3, 10, 1) == 0          # M < 2
    assert ws(100, 1, 10, 50) == 0       # m < 2
    assert ws(100, 513, 10, 50) == 0     # m > 512
    assert ws(100, 512, 10, 50) > 0      # m = 512: the general kernels
    assert ws(100, 3, 0, 50) == 0        # H < 1
    assert ws(100, 3, 10, 101) == 0      # N > M
    assert ws(2**20 + 1, 3, 10, 5) == 0  # M too large
    small = ws(184, 3, 91, 92)
    assert small > 0 and small % 256 == 0
    # the bit-packed dominance matrix dominates: ceil(M/64)^2 * 512 bytes
    big = ws(131072, 10, 2002, 65536)
    mask = (131072 // 64) ** 2 * 512
    assert mask <= big < mask * 1.05


def test_invalid_arguments_enqueue_nothing(lib):
    P = ctypes.c_void_p
    lib.nsga3_select.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_uint64, P, P, P, P, P, ctypes.c_size_t, P]
    assert lib.nsga3_select(None, 10, 3, None, 5, 5, 0, None, None, None, None, None, 0, None) == -1
    fake = P(4096)  # never dereferenced: validation fails first
    # ws too small
    assert lib.nsga3_select(fake, 10, 3, fake, 5, 5, 0, fake, None, None, None, fake, 16, None) == -2
    # misaligned workspace
    assert lib.nsga3_select(fake, 10, 3, fake, 5, 5, 0, fake, None, None, None, P(4100), 1 << 30,
                            None) == -1
    # m out of range
    assert lib.nsga3_select(fake, 10, 513, fake, 5, 5, 0, fake, None, None, None, fake, 1 << 30,
                            None) == -1


def test_noalloc_validates_before_enqueue(lib):
    P, i32 = ctypes.c_void_p, ctypes.c_int32
    f = lib.nsga3_select_noalloc
    f.argtypes = [P, i32, i32, P, i32, i32, ctypes.c_uint64, P, P, P, P, P, P]
    assert f(None, 10, 3, None, 5, 5, 0, None, None, None, None, None, None) == -1
    fake = P(4096)  # never dereferenced: validation fails first
    assert f(fake, 10, 513, fake, 5, 5, 0, fake, None, None, None, None, None) == -1
    assert f(fake, 10, 3, fake, 5, 5, 0, fake, None, None, None, P(4098), None) == -1  # status
    # beyond the 64 MiB scratch (m = 3, M = 30000 needs about 109 MiB)
    assert lib.nsga3_workspace_bytes(30000, 3, 5, 15000) > 64 << 20
    assert f(fake, 30000, 3, fake, 5, 15000, 0, fake, None, None, None, None, None) == -2
    src = open(HEADER).read()
    assert "#define NSGA3_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)" in src


class _Inst(ctypes.Structure):
    _fields_ = [("F", ctypes.c_void_p), ("Z", ctypes.c_void_p), ("selected", ctypes.c_void_p),
                ("rank", ctypes.c_void_p), ("pi", ctypes.c_void_p), ("dist", ctypes.c_void_p),
                ("M", ctypes.c_int32), ("m", ctypes.c_int32), ("H", ctypes.c_int32),
                ("N", ctypes.c_int32), ("seed", ctypes.c_uint64), ("tile", ctypes.c_int32 * 4),
                ("ws", ctypes.c_void_p), ("ws_bytes", ctypes.c_size_t)]


def _batch(shapes, tiles=None):
    arr = (_Inst * len(shapes))()
    for b, (M, m, H, N) in enumerate(shapes):
        arr[b].M, arr[b].m, arr[b].H, arr[b].N = M, m, H, N
        for i, t in enumerate((tiles or {}).get(b, [])):
            arr[b].tile[i] = t
    return arr


def test_instance_struct_matches_header():
    # six pointers, four int32, a uint64, int32[4], a pointer and a size
    assert ctypes.sizeof(_Inst) == 104
    src = open(os.path.join(ROOT, "include", "nsga3.h")).read()
    body = src[src.index("typedef struct nsga3_instance"):src.index("} nsga3_instance;")]
    fields = [ln.split(";")[0].split()[-1].lstrip("*") for ln in body.splitlines()[1:] if ";" in ln]
    names = []
    for f in fields:
        names += [x.strip().lstrip("*") for x in f.split(",")]
    assert names[:6] == ["F", "Z", "selected", "rank", "pi", "dist"]


def test_batched_workspace_bytes(lib):
    f = lib.nsga3_batched_workspace_bytes
    f.restype = ctypes.c_size_t
    f.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    one = _batch([(5000, 3, 91, 2500)])
    # a batch of one holds what the plain call needs
    assert f(one, 1) == lib.nsga3_workspace_bytes(5000, 3, 91, 2500)
    two = _batch([(5000, 3, 91, 2500), (300, 10, 220, 150)])
    assert f(two, 2) > f(one, 1) + lib.nsga3_workspace_bytes(300, 10, 220, 150) // 2
    assert f(two, 0) == 0
    assert f(None, 1) == 0
    assert f(_batch([(5000, 3, 91, 2500)] * 2), 1025) == 0        # B above the limit
    assert f(_batch([(1, 3, 91, 1)]), 1) == 0                     # bad shape
    for t in ([(1 << 30) + 1], [0, 7], [0, 0, 1], [0, 0, 0, 2], [-1], [0, 96]):
        assert f(_batch([(5000, 3, 91, 2500)], {0: t}), 1) == 0, t
    for t in ([1], [3], [65, 16], [0, 91], [8, 80], [1 << 30]):
        assert f(_batch([(5000, 3, 91, 2500)], {0: t}), 1) > 0, t


def test_batched_select_validates_before_enqueue(lib):
    P = ctypes.c_void_p
    lib.nsga3_select_batched.argtypes = [P, ctypes.c_int32, P, ctypes.c_size_t, P]
    arr = _batch([(5000, 3, 91, 2500)])
    # null pointers in the instance
    assert lib.nsga3_select_batched(arr, 1, P(4096), 1 << 30, None) == -1
    fake = 4096
    arr[0].F = arr[0].Z = arr[0].selected = fake
    assert lib.nsga3_select_batched(arr, 1, P(4096), 16, None) == -2      # ws too small
    assert lib.nsga3_select_batched(arr, 1, P(4100), 1 << 30, None) == -1  # misaligned ws
    assert lib.nsga3_select_batched(arr, 0, P(4096), 1 << 30, None) == -1  # empty batch
