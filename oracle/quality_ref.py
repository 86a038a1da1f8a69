"""Reference quality indicators (TEST INFRASTRUCTURE ONLY).

Plain numpy restatements of the two indicators the paper reports for its
runs, used to check the device versions; only the test-suite and bench.py's
reporting may use them, and they share no code with the HIP library.

IGD (inverted generational distance; Sec. IV, the population-size study):
the mean over the points r of a known optimal front R of the least
Euclidean distance from r to a point of the population, in float64.

Normalized hypervolume (Appendix E): with reference point ref = 1.01 f_max
and ideal point ideal = 0.9 f_min per objective, HV_max is the volume of the
box [ideal, ref] and the reported value is HV / HV_max, i.e. the fraction of
the box that the population weakly dominates. It is estimated here as the
fraction of sample points of the box that some population point weakly
dominates (f_k <= y_k for every k). Sample i, objective k:
  h = sm64(seed ^ sm64(i << 8 | k)), sm64 the SplitMix64 output function
  u = (h >> 40) * 2^-24
  y_k = ideal_k + u * (ref_k - ideal_k), each operation rounded in float32
The dominance decision is taken in float32 on both sides (it decides an
integer count), so the count is exact and the device must match it.
"""
import numpy as np

MASK64 = (1 << 64) - 1


def splitmix64(x):
    """SplitMix64 output function (Steele, Lea & Flood 2014), numpy uint64
    arrays (wrapping arithmetic)."""
    with np.errstate(over="ignore"):
        z = np.asarray(x, dtype=np.uint64) + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def igd(F, R):
    """Mean over rows r of R of min over rows f of F of ||r - f||_2 (float64)."""
    F = np.asarray(F, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    best = np.full(len(R), np.inf)
    for a in range(0, len(F), 4096):
        d = np.sqrt(((R[:, None, :] - F[None, a:a + 4096, :]) ** 2).sum(axis=2))
        best = np.minimum(best, d.min(axis=1))
    return float(best.mean())


def hv_box(fmin, fmax):
    """The paper's box: ideal = 0.9 f_min, ref = 1.01 f_max (float32)."""
    return (np.float32(0.9) * np.asarray(fmin, np.float32),
            np.float32(1.01) * np.asarray(fmax, np.float32))


def hv_samples(ideal, ref, samples, seed, start=0):
    """Sample points start .. start + samples - 1 of the box, float32 [s][m]."""
    ideal = np.asarray(ideal, np.float32)
    ref = np.asarray(ref, np.float32)
    m = len(ideal)
    i = np.arange(start, start + samples, dtype=np.uint64)[:, None]
    k = np.arange(m, dtype=np.uint64)[None, :]
    h = splitmix64(np.uint64(seed) ^ splitmix64((i << np.uint64(8)) | k))
    u = (h >> np.uint64(40)).astype(np.float32) * np.float32(2.0 ** -24)
    span = ref - ideal                      # float32 subtraction
    return ideal + u * span                 # float32 product, then float32 sum


def hv_count(F, ideal, ref, samples, seed, chunk=8192):
    """Number of sample points that some row of F weakly dominates."""
    F = np.asarray(F, np.float32)
    count = 0
    for a in range(0, samples, chunk):
        y = hv_samples(ideal, ref, min(chunk, samples - a), seed, start=a)
        covered = np.zeros(len(y), bool)
        for b in range(0, len(F), 512):
            dom = np.all(F[None, b:b + 512, :] <= y[:, None, :], axis=2)
            covered |= dom.any(axis=1)
        count += int(covered.sum())
    return count
