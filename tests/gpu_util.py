"""Helpers for the GPU parity tests (no method arithmetic beyond what the
tolerance checks need)."""
import numpy as np
import pytest
import torch


def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def to_dev(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def to_np(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def perp_dist64(Fn, Z, idx_f, idx_ref):
    """FP64 perpendicular distance of rows Fn[idx_f] to references Z[idx_ref]."""
    W = Z.astype(np.float64)
    W = W / np.linalg.norm(W, axis=1, keepdims=True)
    f = Fn[idx_f].astype(np.float64)
    w = W[idx_ref]
    p = np.sum(f * w, axis=1, keepdims=True)
    return np.linalg.norm(f - p * w, axis=1)


def association_report(Fn64, Z, st, pi_gpu, pi_ref, d_gpu, d_ref, band=1e-6):
    """Compare association on rows st: returns (n_mismatch, n_flagged_near_tie,
    max |d_gpu - d_ref| / ||f||). A mismatch is accepted only when the FP64
    distances of the two references differ by at most band * ||f||."""
    mis = st[pi_gpu[st] != pi_ref[st]]
    norms = np.linalg.norm(Fn64[st].astype(np.float64), axis=1)
    derr = np.abs(d_gpu[st].astype(np.float64) - d_ref[st]) / np.maximum(norms, 1e-30)
    if len(mis):
        dg = perp_dist64(Fn64, Z, mis, pi_gpu[mis])
        dr = perp_dist64(Fn64, Z, mis, pi_ref[mis])
        gap = np.abs(dg - dr) / np.maximum(np.linalg.norm(Fn64[mis], axis=1), 1e-30)
        flagged = int(np.sum(gap <= band))
    else:
        flagged = 0
    return len(mis), flagged, float(derr.max()) if len(st) else 0.0


def near_tie_points(Fn64, Z, st, band=1e-6, chunk=4096):
    """Number of rows of st whose two nearest references (FP64 perpendicular
    distance) are within band * ||f||: the only rows at which an FP32
    association may pick another reference than the FP64 one."""
    W = Z.astype(np.float64)
    W = W / np.linalg.norm(W, axis=1, keepdims=True)
    n = 0
    for a in range(0, len(st), chunk):
        f = Fn64[st[a:a + chunk]].astype(np.float64)
        nf = np.linalg.norm(f, axis=1)
        p = f @ W.T
        d = np.sqrt(np.maximum(nf[:, None] ** 2 - p * p, 0.0))
        two = np.partition(d, 1, axis=1)[:, :2] if d.shape[1] > 1 else np.concatenate([d, d + np.inf], 1)
        n += int(np.sum(np.abs(two[:, 1] - two[:, 0]) <= band * (1 + 1e-6) * np.maximum(nf, 1e-30)))
    return n


def front_info_of(rank, N):
    """front_info = (l, |S|, K, l + 1) implied by 0-based ranks and N."""
    ranked = rank[rank != 0x7FFFFFFF]
    l = int(ranked.max())
    s = int(np.sum(ranked < l))
    return np.array([l, s, N - s, l + 1], np.int32)


def asf64(F, z, x, k):
    """FP64 achievement scalarizing value of point x for axis k (weights 1 on
    k, 1e-6 elsewhere, i.e. 1e6 times the other translated objectives)."""
    fp = F[x].astype(np.float64) - z
    g = 1e6 * fp
    g[k] = fp[k]
    return g.max()


def select_parity(inst, g, dev):
    """End-to-end parity of one selection `g` (dict of numpy selected, rank,
    pi, dist from the GPU) against the FP64 oracle:
      - ranks bit-exact;
      - extreme points equal to the oracle's, or an FP64 ASF near-tie
        (gap <= 1e-6 relative), counted;
      - when the extremes agree: every pi mismatch against the oracle's FP64
        association is a near-tie (FP64 distance gap <= 1e-6 ||f_n||), and
        |d_gpu - d_oracle| < 1e-6 ||f_n|| for every point of S_t;
      - the selection equals the oracle's niching of the GPU's own
        (rank, pi, dist), always, and the pure-FP64 oracle's selection when
        nothing upstream was flagged.
    Returns dict(ext_ties, pi_ties, dist_err, n_st, identical, st, Fn)."""
    import oracle
    from paper_2504_06067_amd import nsga3

    F, Z, N, seed = inst["F"], inst["Z"], inst["N"], inst["seed"]
    ref = oracle.select(F, Z, N, seed)
    assert np.array_equal(g["rank"], ref["rank"]), "ranks differ from the oracle"
    fi = front_info_of(ref["rank"], N)
    chained = oracle.niche(g["rank"], fi, g["pi"], g["dist"].astype(np.float64), len(Z), N, seed)
    assert np.array_equal(g["selected"], chained), "selection differs from the oracle's niching"
    st = np.where(ref["rank"] <= fi[0])[0]
    nrm = oracle.normalize(F, ref["rank"], fi)
    out = nsga3.normalize(to_dev(F, dev), to_dev(ref["rank"], dev), to_dev(fi, dev))
    ext = to_np(out["extreme"])
    ext_ties = 0
    for k in range(F.shape[1]):
        if ext[k] != nrm["extreme"][k]:
            a = asf64(F, nrm["ideal"], ext[k], k)
            b = asf64(F, nrm["ideal"], nrm["extreme"][k], k)
            assert abs(a - b) <= 1e-6 * max(abs(b), 1e-30), ("extreme point", k, a, b)
            ext_ties += 1
    pi_ties, derr = 0, 0.0
    if ext_ties == 0:
        Fn = np.nan_to_num(nrm["Fn"], nan=0.0)
        nmis, pi_ties, derr = association_report(Fn, Z, st, g["pi"], ref["pi"], g["dist"],
                                                 ref["dist"])
        assert nmis == pi_ties, f"{nmis - pi_ties} association mismatches outside the near-tie band"
        assert derr < 1e-6, derr
    identical = bool(np.array_equal(g["selected"], ref["selected"]))
    if ext_ties == 0 and pi_ties == 0:
        assert identical, "selection differs from the FP64 oracle with nothing flagged"
    return dict(ext_ties=ext_ties, pi_ties=pi_ties, dist_err=derr, n_st=len(st),
                identical=identical, st=st, Fn=np.nan_to_num(nrm["Fn"], nan=0.0))
