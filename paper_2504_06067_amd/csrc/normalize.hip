// Normalization of S_t (Algorithm 1 "associate ... using normalized
// objectives"; Algorithm 2 "Normalize"), following the Deb & Jain 2014
// procedure that the paper cites: ideal point, ASF extreme points, hyperplane
// intercepts (the one FP64 step: an m x m pivoted elimination), and the
// per-objective maximum as the fallback when the hyperplane is degenerate.
// For a batch of independent instances.
//
// Kernels:
//   k_norm_reduce   per-objective min (ideal) and max over S_t; builds the
//                   S_t index list (order irrelevant to every result); in a
//                   whole selection also prepares the association outputs
//   k_norm_extreme  per-axis ASF argmin over S_t as a 64-bit (value, index) min
//   k_norm_solve    one wave per instance: FP64 elimination, degeneracy tests
//   k_norm_apply    Fn = (f - z) * (1 / a) over S_t
#include "nsga3_internal.h"

namespace nsga3 {

__global__ __launch_bounds__(256) void k_norm_reduce(BatchView bv) {
    const Local L = locate(bv.pt_pref, bv.B);
    CInst &I = bv.tab[L.b];
    const int x = L.i, M = I.M, m = I.m;
    Ctrl *ctrl = I.P.ctrl;
    const int l = I.front_info[0];
    const bool in = x < M && I.rank[x] >= 0 && I.rank[x] <= l;
    if ((bv.run & RUN_ASSOC) && x < M) {
        // the association reuses this list; rows outside S_t get pi = dist = -1
        if (in) I.P.akey[x] = ~0ull;
        else {
            I.pi[x] = -1;
            I.dist[x] = -1.0f;
        }
    }
    const u64 bal = ballot(in);
    if (bal == 0) return;
    const int lane = lane_id();
    int base = 0;
    if (lane == 0) base = atomicAdd(&ctrl->list_count, __popcll(bal));
    base = __shfl(base, 0, 64);
    if (in) I.P.list[base + mbcnt(bal)] = x;
    for (int k = 0; k < m; ++k) {
        const float v = in ? I.F[(size_t)x * m + k] : 0.0f;
        const unsigned lo = wave_min_u32(in ? f2ord(v) : 0xffffffffu);
        const unsigned hi = wave_max_u32(in ? f2ord(v) : 0u);
        if (lane == 0) {
            atomicMin(&ctrl->zmin_enc[k], lo);
            atomicMax(&ctrl->fmax_enc[k], hi);
        }
    }
}

// ASF_k(x) = max(f'_k, max_{j != k} 1e6 * f'_j) with f' = f - z >= 0 on S_t,
// so the raw float bits order like the values; ties go to the least index.
// Grid: padded points of the group's instances (one launch per m).
template <int MO>
__global__ __launch_bounds__(256) void k_norm_extreme(BatchView bv, int gs, int gn, int pt0) {
    const int base = uniform(pt0 + (int)(blockIdx.x * blockDim.x));
    const int gi = uniform(find_range(bv.pt_pref, bv.B, base));
    CInst &I = bv.tab[gi];
    Ctrl *ctrl = I.P.ctrl;
    const int n = ctrl->list_count;
    const int i = base - bv.pt_pref[gi] + (int)threadIdx.x;
    if (base - bv.pt_pref[gi] >= n || I.m != MO) return;
    const bool in = i < n;
    const int x = in ? I.P.list[i] : 0;
    float fp[MO], g[MO];
#pragma unroll
    for (int k = 0; k < MO; ++k) {
        const float z = ord2f(ctrl->zmin_enc[k]);
        fp[k] = in ? I.F[(size_t)x * MO + k] - z : 0.0f;
        g[k] = 1e6f * fp[k];
    }
    // largest and second largest of g, with the position of the largest
    float g1 = g[0], g2 = -INFINITY;
    int p1 = 0;
#pragma unroll
    for (int k = 1; k < MO; ++k) {
        if (g[k] > g1) { g2 = g1; g1 = g[k]; p1 = k; }
        else if (g[k] > g2) g2 = g[k];
    }
#pragma unroll
    for (int k = 0; k < MO; ++k) {
        const float other = (k == p1) ? g2 : g1;
        const float asf = fmaxf(fp[k], other);
        u64 key = in ? (((u64)__float_as_uint(asf) << 32) | (unsigned)x) : ~0ull;
        key = wave_min_u64(key);
        if (lane_id() == 0 && key != ~0ull) atomicMin(&ctrl->ext_key[k], key);
    }
    (void)gs;
    (void)gn;
}

// One wave per instance; lane 0 does the elimination: E[k][j] = f(e_k)_j - z_j
// in FP64; solve E b = 1 by Gaussian elimination with partial pivoting
// (largest |pivot|, least row on ties); a_k = 1 / b_k unless degenerate.
__global__ void k_norm_solve(BatchView bv) {
    CInst &I = bv.tab[blockIdx.x];
    if (threadIdx.x != 0) return;
    Ctrl *ctrl = I.P.ctrl;
    const int M = I.M, m = I.m;
    double z[NSGA3_MAX_OBJECTIVES], fmx[NSGA3_MAX_OBJECTIVES], b[NSGA3_MAX_OBJECTIVES];
    double A[NSGA3_MAX_OBJECTIVES][NSGA3_MAX_OBJECTIVES], r[NSGA3_MAX_OBJECTIVES];
    double colmax[NSGA3_MAX_OBJECTIVES];
    int ext[NSGA3_MAX_OBJECTIVES];
    int degen = 0;
    for (int k = 0; k < m; ++k) {
        const float zf = ord2f(ctrl->zmin_enc[k]);
        z[k] = (double)zf;
        fmx[k] = (double)ord2f(ctrl->fmax_enc[k]) - z[k];
        ext[k] = (int)(unsigned)(ctrl->ext_key[k] & 0xffffffffull);
        if (ext[k] < 0 || ext[k] >= M) { ext[k] = 0; degen = 1; atomicOr(&ctrl->status, ST_INTERNAL); }
        ctrl->zf[k] = zf;
        I.ideal[k] = zf;
        I.extreme[k] = ext[k];
    }
    for (int i = 0; i < m; ++i) {
        r[i] = 1.0;
        for (int j = 0; j < m; ++j) A[i][j] = (double)I.F[(size_t)ext[i] * m + j] - z[j];
    }
    for (int j = 0; j < m; ++j) {
        colmax[j] = 0.0;
        for (int i = 0; i < m; ++i) colmax[j] = fmax(colmax[j], fabs(A[i][j]));
    }
    for (int c = 0; c < m && !degen; ++c) {
        int piv = c;
        for (int i = c + 1; i < m; ++i)
            if (fabs(A[i][c]) > fabs(A[piv][c])) piv = i;
        if (colmax[c] == 0.0 || fabs(A[piv][c]) < 1e-10 * colmax[c]) { degen = 1; break; }
        if (piv != c) {
            for (int j = 0; j < m; ++j) { double t = A[c][j]; A[c][j] = A[piv][j]; A[piv][j] = t; }
            double t = r[c]; r[c] = r[piv]; r[piv] = t;
        }
        for (int i = c + 1; i < m; ++i) {
            const double f = A[i][c] / A[c][c];
            for (int j = c; j < m; ++j) A[i][j] = __dsub_rn(A[i][j], __dmul_rn(f, A[c][j]));
            r[i] = __dsub_rn(r[i], __dmul_rn(f, r[c]));
        }
    }
    if (!degen) {
        for (int i = m - 1; i >= 0; --i) {
            double s = r[i];
            for (int j = i + 1; j < m; ++j) s = __dsub_rn(s, __dmul_rn(A[i][j], b[j]));
            b[i] = s / A[i][i];
        }
    }
    double a[NSGA3_MAX_OBJECTIVES];
    for (int k = 0; k < m && !degen; ++k) {
        if (!(b[k] > 0.0)) { degen = 1; break; }
        a[k] = 1.0 / b[k];
        if (!isfinite(a[k]) || a[k] < 1e-6 * fmx[k]) { degen = 1; break; }
    }
    if (degen)
        for (int k = 0; k < m; ++k) a[k] = fmx[k] > 0.0 ? fmx[k] : 1.0;
    for (int k = 0; k < m; ++k) {
        I.intercept[k] = a[k];
        ctrl->recip[k] = (float)(1.0 / a[k]);
    }
    *I.degenerate = degen;
}

__global__ __launch_bounds__(256) void k_norm_apply(BatchView bv) {
    const Local L = locate(bv.pt_pref, bv.B);
    CInst &I = bv.tab[L.b];
    const Ctrl *ctrl = I.P.ctrl;
    const int n = ctrl->list_count;
    if (L.i >= n) return;
    const int x = I.P.list[L.i], m = I.m;
    for (int k = 0; k < m; ++k)
        I.Fn[(size_t)x * m + k] = (I.F[(size_t)x * m + k] - ctrl->zf[k]) * ctrl->recip[k];
}

hipError_t launch_normalize(const HostPlan &hp, const BatchView &bv, hipStream_t s) {
    const unsigned pblocks = (unsigned)(hp.npt / 256);
    NSGA3_LAUNCH("norm_reduce", k_norm_reduce, dim3(pblocks), dim3(256), 0, s, bv);
    for (int g = 0; g < hp.ngroups; ++g) {
#define NSGA3_EXT_CASE(MO)                                                                     \
    case MO:                                                                                   \
        NSGA3_LAUNCH("norm_extreme", k_norm_extreme<MO>, dim3(pblocks), dim3(256), 0, s, bv,   \
                     hp.grp_start[g], hp.grp_start[g + 1] - hp.grp_start[g], 0);               \
        break;
        switch (hp.grp_m[g]) {
            NSGA3_EXT_CASE(2) NSGA3_EXT_CASE(3) NSGA3_EXT_CASE(4) NSGA3_EXT_CASE(5)
            NSGA3_EXT_CASE(6) NSGA3_EXT_CASE(7) NSGA3_EXT_CASE(8) NSGA3_EXT_CASE(9)
            NSGA3_EXT_CASE(10) NSGA3_EXT_CASE(11) NSGA3_EXT_CASE(12) NSGA3_EXT_CASE(13)
            NSGA3_EXT_CASE(14) NSGA3_EXT_CASE(15) NSGA3_EXT_CASE(16)
            default: return hipErrorInvalidValue;
        }
#undef NSGA3_EXT_CASE
    }
    NSGA3_LAUNCH("norm_solve", k_norm_solve, dim3(hp.B), dim3(64), 0, s, bv);
    NSGA3_LAUNCH("norm_apply", k_norm_apply, dim3(pblocks), dim3(256), 0, s, bv);
    return hipGetLastError();
}

}  // namespace nsga3
