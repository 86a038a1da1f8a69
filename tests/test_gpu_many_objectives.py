"""Many objectives (m above the 16 of the specialized kernels, up to 512: the
general dominance, normalization and association kernels), at the paper's
objective-scaling shape (2N = 1600) and smaller ragged ones: ranks
bit-exact; extremes exact or FP64 ASF near-ties; every association mismatch
a near-tie within 1e-6 ||f_n||, the distance within 1e-6 ||f_n||; the
selection equal to the oracle's niching of the GPU's own (rank, pi, dist),
and to the FP64 oracle when nothing is flagged. Intercepts agree with the
oracle's to rounding (the general solve's back substitution sums in another
order)."""
import os

import numpy as np
import pytest

import oracle
from gpu_util import device, near_tie_points, select_parity, to_dev, to_np
from paper_2504_06067_amd import nsga3
from paper_2504_06067_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _oracle_threads():
    oracle.set_threads(min(16, os.cpu_count() or 1))
    yield
    oracle.set_threads(1)


def run(inst, dev):
    out = nsga3.select(to_dev(inst["F"], dev), to_dev(inst["Z"], dev), inst["N"], inst["seed"],
                       intermediates=True)
    return {k: to_np(v) for k, v in out.items()}


@pytest.mark.parametrize("m,p,M,law", [(17, 3, 700, "exp"), (32, 2, 1600, "exp"),
                                       (64, 1, 1600, "cube"), (128, 1, 1600, "exp"),
                                       (512, 1, 1600, "exp"), (200, 1, 333, "cube")])
def test_select_parity(m, p, M, law):
    dev = device()
    print(f"many objectives: m={m} M={M}", flush=True)
    F = wl.objectives(np.random.default_rng(m), M, m, law)
    Z = wl.das_dennis(m, p)
    inst = dict(F=F, Z=Z, N=M // 2, H=len(Z), seed=m)
    r = select_parity(inst, run(inst, dev), dev)
    assert r["ext_ties"] == 0
    # at large m the degenerate intercepts (largest value per objective) put
    # exact 1.0 in several objectives of one point: exact FP64 ties between
    # axis references, which FP32 sums in different orders may break either
    # way. Mismatches are bounded by the near-tie points, never beyond.
    assert r["pi_ties"] <= near_tie_points(r["Fn"], Z, r["st"])
    print(f"m={m}: {r['pi_ties']} flagged association near-ties of {r['n_st']}", flush=True)


@pytest.mark.parametrize("m", [24, 96])
def test_many_fronts(m):
    """Levels of three points each (every objective at the level, plus 0.5 in
    one objective chosen per point): points of one level are incomparable,
    every lower level dominates every higher one, so the fronts are the
    levels, 150 of them before N is reached."""
    dev = device()
    rng = np.random.default_rng(m)
    M = 900
    level = rng.permutation(M) // 3
    F = np.repeat(level.astype(np.float32)[:, None], m, axis=1)
    F[np.arange(M), rng.integers(0, m, M)] += 0.5
    Z = wl.das_dennis(m, 1)
    inst = dict(F=F, Z=Z, N=M // 2, H=len(Z), seed=5)
    g = run(inst, dev)
    ref = oracle.select(F, Z, M // 2, 5)
    assert np.array_equal(g["rank"], ref["rank"])
    assert int(g["rank"][g["rank"] != nsga3.UNRANKED].max()) == 149
    r = select_parity(inst, g, dev)
    assert r["pi_ties"] <= near_tie_points(r["Fn"], Z, r["st"])


@pytest.mark.parametrize("m", [20, 64, 300])
def test_normalize_intercepts(m):
    dev = device()
    rng = np.random.default_rng(m)
    E = 1e-7 * rng.random((m, m)) + np.diag(1.0 + rng.random(m))
    zero_rest = np.zeros(m)
    zero_rest[0] = 3.0
    zero_first = np.full(m, 3.0)
    zero_first[0] = 0.0
    F = np.concatenate([E, [zero_rest, zero_first], 0.5 + rng.random((60, m))]).astype(np.float32)
    rank = np.zeros(len(F), np.int32)
    fi = np.array([0, 0, len(F), 1], np.int32)
    ref = oracle.normalize(F, rank, fi)
    out = nsga3.normalize(to_dev(F, dev), to_dev(rank, dev), to_dev(fi, dev))
    assert np.array_equal(to_np(out["ideal"]).astype(np.float64), ref["ideal"])
    assert np.array_equal(to_np(out["extreme"]), ref["extreme"])
    assert int(to_np(out["degenerate"])[0]) == ref["degenerate"] == 0
    np.testing.assert_allclose(to_np(out["intercept"]), ref["intercept"], rtol=1e-12)
    Fn = to_np(out["Fn"]).astype(np.float64)
    err = np.abs(Fn - ref["Fn"]) / np.linalg.norm(ref["Fn"], axis=1, keepdims=True)
    assert err.max() < 2e-6


def test_normalize_degenerate():
    dev = device()
    rng = np.random.default_rng(9)
    x = rng.random((90, 20))
    F = np.concatenate([x, x[:, :1]], axis=1).astype(np.float32)  # objective 21 = objective 1
    rank = np.zeros(90, np.int32)
    fi = np.array([0, 0, 90, 1], np.int32)
    ref = oracle.normalize(F, rank, fi)
    out = nsga3.normalize(to_dev(F, dev), to_dev(rank, dev), to_dev(fi, dev))
    assert ref["degenerate"] == 1 == int(to_np(out["degenerate"])[0])
    assert np.array_equal(to_np(out["intercept"]), ref["intercept"])


@pytest.mark.parametrize("m,p", [(40, 1), (128, 1), (33, 2)])
def test_points_on_reference_directions(m, p):
    dev = device()
    Z = wl.das_dennis(m, p)
    H = len(Z)
    c = np.random.default_rng(m).uniform(0.5, 2.0, H)
    Fn = (Z.astype(np.float64) / np.linalg.norm(Z.astype(np.float64), axis=1, keepdims=True)
          * c[:, None]).astype(np.float32)
    rank = np.zeros(H, np.int32)
    fi = np.array([0, 0, H, 1], np.int32)
    pi, d = nsga3.associate(to_dev(Fn, dev), to_dev(rank, dev), to_dev(fi, dev), to_dev(Z, dev))
    assert np.array_equal(to_np(pi), np.arange(H))
    assert np.all(to_np(d) < 1e-6 * np.linalg.norm(Fn, axis=1))


def test_mixed_batch_equals_plain():
    """Instances of specialized and general m in one batched call give what
    each gives alone."""
    dev = device()
    shapes = [(800, 3, 12), (600, 40, 1), (1000, 10, 3), (500, 300, 1)]
    probs, plain = [], []
    for i, (M, m, p) in enumerate(shapes):
        F = wl.objectives(np.random.default_rng(i), M, m, "exp")
        Z = wl.das_dennis(m, p)
        probs.append(dict(F=to_dev(F, dev), Z=to_dev(Z, dev), N=M // 2, seed=i))
        plain.append(run(dict(F=F, Z=Z, N=M // 2, seed=i), dev))
    bt = nsga3.Batch(probs, intermediates=True)
    bt.run()
    assert bt.status() == [nsga3.OK] * len(shapes)
    for b in range(len(shapes)):
        for k in ("selected", "rank", "pi", "dist"):
            assert np.array_equal(to_np(getattr(bt, k)[b]), plain[b][k]), (b, k)
