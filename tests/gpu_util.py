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
