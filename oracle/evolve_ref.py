"""Reference of the served generation step (TEST INFRASTRUCTURE ONLY).

Plain float64 numpy restatement of the offspring generation that a served
run repeats between selections: random mating, simulated binary crossover
(SBX) and polynomial mutation, the variation operators the paper names for
the offspring stage (Sec. II-C; Algorithm 1, "Crossover+Mutation"), followed
by a synthetic objective map. Only the test-suite may use it; it shares no
code with the HIP library.

Definitions (the GPU path implements the same ones in float32):
  h(seed, g, tag, i, j) = sm64(seed ^ sm64(tag << 58 | (g mod 2^16) << 42 |
                          (j mod 2^10) << 32 | i)), sm64 = SplitMix64 output
  u01(h) = (h >> 40) * 2^-24, an index below n is h mod n
  tags: 4 initial value, 5 / 6 first / second parent, 7 SBX, 8 mutation
        applied?, 9 mutation draw
  SBX (Deb & Agrawal 1995), distribution index eta = 20, on every variable:
      beta = (2u)^(1/(eta+1))              if u <= 1/2
             (1 / (2(1-u)))^(1/(eta+1))    otherwise
      c1 = ((1+beta) x1 + (1-beta) x2) / 2,  c2 = ((1-beta) x1 + (1+beta) x2) / 2
  polynomial mutation (Deb & Goyal 1996), rate 1/d (as float32), index 20,
  range 1:
      delta = (2u)^(1/(eta+1)) - 1         if u < 1/2
              1 - (2(1-u))^(1/(eta+1))     otherwise
  every variable is clamped to [0, 1 - 2^-24] after crossover and again after
  mutation.
  objective map: y = A (x_1..x_{d-1} - 1/2), u = |y| / ||y|| (1/sqrt(m) when
  y = 0), f = u (1 - 0.3 ln(1 - x_d)).
"""
import numpy as np

MASK64 = (1 << 64) - 1
XMAX = 1.0 - 2.0 ** -24
ETA_C = 20.0
ETA_M = 20.0
TAG_INIT, TAG_PA, TAG_PB, TAG_SBX, TAG_PM_APPLY, TAG_PM_U = 4, 5, 6, 7, 8, 9


def splitmix64(x):
    """SplitMix64 output function (Steele, Lea & Flood 2014), Python ints."""
    z = (x + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def h(seed, g, tag, i, j):
    c = (tag << 58) | ((g & 0xFFFF) << 42) | ((j & 0x3FF) << 32) | (i & 0xFFFFFFFF)
    return splitmix64((seed & MASK64) ^ splitmix64(c))


def u01(hv):
    return (hv >> 40) * 2.0 ** -24


def sbx_beta(u):
    e = 1.0 / (ETA_C + 1.0)
    return (2.0 * u) ** e if u <= 0.5 else (1.0 / (2.0 * (1.0 - u))) ** e


def pm_delta(u):
    e = 1.0 / (ETA_M + 1.0)
    return (2.0 * u) ** e - 1.0 if u < 0.5 else 1.0 - (2.0 * (1.0 - u)) ** e


def pm_threshold(d):
    """Mutation rate 1/d as the float32 value that the GPU compares against
    (the decision to mutate is taken in the same precision on both sides)."""
    return float(np.float32(1.0) / np.float32(d))


def clamp(x):
    return min(max(x, 0.0), XMAX)


def objectives(X, A):
    """f for every row of X [n][d] (float64), A [m][d-1]."""
    X = np.asarray(X, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    m = A.shape[0]
    y = (X[:, :-1] - 0.5) @ A.T
    n = np.linalg.norm(y, axis=1, keepdims=True)
    u = np.where(n > 0, np.abs(y) / np.where(n > 0, n, 1.0), 1.0 / np.sqrt(m))
    rad = 1.0 - 0.3 * np.log(1.0 - X[:, -1])
    return u * rad[:, None]


def init_population(N, d, seed):
    X = np.empty((N, d))
    for i in range(N):
        for j in range(d):
            X[i, j] = u01(h(seed, 0, TAG_INIT, i, j))
    return X


def offspring(P, seed, g):
    """N offspring of population P [N][d] (float64) at generation g."""
    N, d = P.shape
    O = np.empty((N, d))
    for i in range(N):
        k = i >> 1
        a = h(seed, g, TAG_PA, k, 0) % N
        b = h(seed, g, TAG_PB, k, 0) % N
        for j in range(d):
            x1, x2 = P[a, j], P[b, j]
            beta = sbx_beta(u01(h(seed, g, TAG_SBX, k, j)))
            if i & 1:
                y = 0.5 * ((1.0 - beta) * x1 + (1.0 + beta) * x2)
            else:
                y = 0.5 * ((1.0 + beta) * x1 + (1.0 - beta) * x2)
            y = clamp(y)
            if u01(h(seed, g, TAG_PM_APPLY, i, j)) < pm_threshold(d):
                y = clamp(y + pm_delta(u01(h(seed, g, TAG_PM_U, i, j))))
            O[i, j] = y
    return O
