"""The point placement that the dominance and peel kernels rely on, checked on
the CPU by brute force (the kernels themselves are checked end to end by the
GPU parity tests).

The library places points in ascending buckets of the first objective,
bucket(x) = floor((f_1(x) - lo) * B / (hi - lo)) clamped to [0, B), computed
in float32. The kernels then treat a tile (column block ib, row block jb) as
ordered when ib < row_ord[jb] and compute only "i dominates j" there, and the
peel reads column block c's words only from row blocks below col_end[c]. These
tests restate the placement with numpy and check the claims the kernels need:
  * a point is never dominated by a point in a higher bucket;
  * in an ordered tile every column point has a smaller f_1 than every row
    point (so "j dominates i" is empty and f_1 needs no compare);
  * every word the peel reads (w < col_end[c]) is written by the dominance
    kernel, and every word it skips holds no dominator.
"""
import numpy as np
import pytest

B = 1024  # buckets (PLACE_BUCKETS)


def buckets(f1):
    f1 = np.asarray(f1, np.float32)
    lo, hi = f1.min(), f1.max()
    with np.errstate(over="ignore", invalid="ignore"):
        span = np.float32(hi - lo)
        scale = np.float32(B) / span if (span > 0 and np.isfinite(span)) else np.float32(0)
        t = (f1 - lo) * scale
    return np.where(t >= B, B - 1, np.where(t > 0, np.floor(np.nan_to_num(t)), 0)).astype(np.int64)


def place(F):
    """Positions in ascending bucket order (ties in any order: here by index),
    with row_ord and col_end as the scatter kernel writes them."""
    M = len(F)
    b = buckets(F[:, 0])
    perm = np.argsort(b, kind="stable")
    start = np.concatenate([[0], np.cumsum(np.bincount(b, minlength=B))])
    W = (M + 63) // 64
    bs = b[perm]
    row_ord = np.array([start[bs[64 * jb]] >> 6 for jb in range(W)])
    col_end = np.array([(start[bs[min(64 * c + 63, M - 1)] + 1] + 63) >> 6 for c in range(W)])
    return perm, b, row_ord, col_end


def dominates(F):
    """D[i, j] = point i dominates point j (minimization, float32 compares)."""
    le = np.all(F[:, None, :] <= F[None, :, :], axis=2)
    lt = np.any(F[:, None, :] < F[None, :, :], axis=2)
    return le & lt


def cases():
    rng = np.random.default_rng(3)
    yield "continuous", rng.random((700, 3)).astype(np.float32)
    yield "grid_ties", rng.integers(0, 5, (650, 4)).astype(np.float32)
    yield "negative", (rng.standard_normal((300, 2)) * 1e3).astype(np.float32)
    z = rng.random((260, 3)).astype(np.float32)
    z[::3, 0] = -0.0
    z[1::3, 0] = 0.0
    yield "signed_zero", z
    yield "all_equal", np.ones((200, 3), np.float32)
    e = rng.random((330, 3)).astype(np.float32)
    e[0, 0], e[1, 0] = -3.0e38, 3.0e38  # span overflows: one bucket
    yield "huge_span", e
    t = rng.random((129, 5)).astype(np.float32)
    t[:, 0] = np.float32(1.0) + np.arange(129, dtype=np.float32) * np.float32(2.0 ** -23)
    yield "narrow_range", t  # consecutive floats in f_1


@pytest.mark.parametrize("name,F", list(cases()), ids=[c[0] for c in cases()])
def test_lower_bucket_never_dominated_by_higher(name, F):
    b = buckets(F[:, 0])
    D = dominates(F)
    i, j = np.nonzero(D)  # i dominates j
    assert np.all(b[i] <= b[j]), name


@pytest.mark.parametrize("name,F", list(cases()), ids=[c[0] for c in cases()])
def test_ordered_tiles_and_peel_bounds(name, F):
    M = len(F)
    perm, b, row_ord, col_end = place(F)
    W = len(row_ord)
    P = F[perm]                      # objectives by position
    bp = b[perm]
    D = dominates(P)                 # by position
    blocks = [np.arange(64 * w, min(64 * w + 64, M)) for w in range(W)]
    for jb in range(W):
        assert 0 <= row_ord[jb] <= jb
        for ib in range(row_ord[jb]):
            ci, rj = blocks[ib], blocks[jb]
            # ordered: every column point has a smaller bucket, hence f_1
            assert bp[ci].max() < bp[rj].min()
            assert P[ci, 0].max() < P[rj, 0].min()
            # no row point dominates a column point
            assert not D[np.ix_(rj, ci)].any()
    for c in range(W):
        assert c + 1 <= col_end[c] <= W
        for w in range(col_end[c], W):
            # skipped words: no point of block w dominates a point of block c
            assert not D[np.ix_(blocks[w], blocks[c])].any()
        for w in range(c + 1, col_end[c]):
            # read words above the diagonal come from full tiles (c, w),
            # whose reverse words the dominance kernel writes
            assert c >= row_ord[w]


def test_ordered_share_of_paper_workloads():
    """Most tiles are ordered on the synthetic workloads (so the kernel's
    cheap path carries the work); the threshold is loose on purpose."""
    from paper_2504_06067_amd import workloads as wl
    q = wl.plain_instance("large", 0)
    perm, b, row_ord, col_end = place(q["F"])
    W = len(row_ord)
    assert row_ord.sum() / (W * (W + 1) / 2) > 0.9
