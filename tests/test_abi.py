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
    assert ws(100, 17, 10, 50) == 0      # m > 16
    assert ws(100, 3, 0, 50) == 0        # H < 1
    assert ws(100, 3, 10, 101) == 0      # N > M
    assert ws(2**20 + 1, 3, 10, 5) == 0  # M too large
    small = ws(184, 3, 91, 92)
    assert small > 0 and small % 256 == 0
    # the bit-packed dominance matrix dominates: ceil(M/64)^2 * 512 bytes, held
    # twice (word-major as computed, row-major for the peel's scans)
    big = ws(131072, 10, 2002, 65536)
    mask = (131072 // 64) ** 2 * 512
    assert 2 * mask <= big < 2 * mask * 1.05


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
    assert lib.nsga3_select(fake, 10, 17, fake, 5, 5, 0, fake, None, None, None, fake, 1 << 30,
                            None) == -1
