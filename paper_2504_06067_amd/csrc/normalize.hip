// Normalization of S_t (Algorithm 1 "associate ... using normalized
// objectives"; Algorithm 2 "Normalize"), following the Deb & Jain 2014
// procedure that the paper cites: ideal point, ASF extreme points, hyperplane
// intercepts (the one FP64 step: an m x m pivoted elimination), and the
// per-objective maximum as the fallback when the hyperplane is degenerate.
//
// Kernels:
//   k_norm_init     resets the reductions
//   k_norm_reduce   per-objective min (ideal) and max over S_t; builds the
//                   S_t index list (order irrelevant to every result)
//   k_norm_extreme  per-axis ASF argmin over S_t as a 64-bit (value, index) min
//   k_norm_solve    one thread: FP64 elimination, degeneracy tests, outputs
//   k_norm_apply    Fn = (f - z) * (1 / a) over S_t
#include "nsga3_internal.h"

namespace nsga3 {

__global__ void k_norm_init(Ctrl *ctrl, int m, bool reset_status) {
    const int t = threadIdx.x;
    if (t == 0) {
        if (reset_status) ctrl->status = 0;
        ctrl->list_count = 0;
    }
    if (t < m) {
        ctrl->zmin_enc[t] = 0xffffffffu;
        ctrl->fmax_enc[t] = 0u;
        ctrl->ext_key[t] = ~0ull;
    }
}

__global__ __launch_bounds__(256) void k_norm_reduce(const float *__restrict__ F,
                                                      const int *__restrict__ rank,
                                                      const int *__restrict__ front_info, int M,
                                                      int m, int *__restrict__ list, Ctrl *ctrl) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int l = front_info[0];
    const bool in = x < M && rank[x] >= 0 && rank[x] <= l;
    const u64 bal = ballot(in);
    if (bal == 0) return;
    const int lane = lane_id();
    int base = 0;
    if (lane == 0) base = atomicAdd(&ctrl->list_count, __popcll(bal));
    base = __shfl(base, 0, 64);
    if (in) list[base + mbcnt(bal)] = x;
    for (int k = 0; k < m; ++k) {
        const float v = in ? F[(size_t)x * m + k] : 0.0f;
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
template <int MO>
__global__ __launch_bounds__(256) void k_norm_extreme(const float *__restrict__ F,
                                                       const int *__restrict__ list, Ctrl *ctrl) {
    const int n = ctrl->list_count;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if ((int)(blockIdx.x * blockDim.x) >= n) return;
    const bool in = i < n;
    const int x = in ? list[i] : 0;
    float fp[MO], g[MO];
#pragma unroll
    for (int k = 0; k < MO; ++k) {
        const float z = ord2f(ctrl->zmin_enc[k]);
        fp[k] = in ? F[(size_t)x * MO + k] - z : 0.0f;
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
}

// Single thread: E[k][j] = f(e_k)_j - z_j in FP64; solve E b = 1 by Gaussian
// elimination with partial pivoting (largest |pivot|, least row on ties);
// a_k = 1 / b_k unless degenerate.
__global__ void k_norm_solve(const float *__restrict__ F, int M, int m, Ctrl *ctrl, float *ideal,
                             double *intercept, int *extreme, int *degenerate) {
    if (threadIdx.x != 0) return;
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
        ideal[k] = zf;
        extreme[k] = ext[k];
    }
    for (int i = 0; i < m; ++i) {
        r[i] = 1.0;
        for (int j = 0; j < m; ++j) A[i][j] = (double)F[(size_t)ext[i] * m + j] - z[j];
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
        intercept[k] = a[k];
        ctrl->recip[k] = (float)(1.0 / a[k]);
    }
    *degenerate = degen;
}

__global__ __launch_bounds__(256) void k_norm_apply(const float *__restrict__ F,
                                                     const int *__restrict__ list, int m,
                                                     float *__restrict__ Fn, const Ctrl *ctrl) {
    const int n = ctrl->list_count;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int x = list[i];
    for (int k = 0; k < m; ++k)
        Fn[(size_t)x * m + k] = (F[(size_t)x * m + k] - ctrl->zf[k]) * ctrl->recip[k];
}

hipError_t launch_normalize(const Layout &L, const Ptrs &P, const float *F, const int *rank,
                            const int *front_info, float *Fn, float *ideal, double *intercept,
                            int *extreme, int *degenerate, bool reset_status, hipStream_t s) {
    const int M = L.M, m = L.m;
    const unsigned blocks = (unsigned)((M + 255) / 256);
    NSGA3_LAUNCH("norm_init", k_norm_init, dim3(1), dim3(64), 0, s, P.ctrl, m, reset_status);
    NSGA3_LAUNCH("norm_reduce", k_norm_reduce, dim3(blocks), dim3(256), 0, s, F, rank, front_info, M, m,
                       P.list, P.ctrl);
#define NSGA3_EXT_CASE(MO)                                                                     \
    case MO:                                                                                   \
        NSGA3_LAUNCH("norm_extreme", k_norm_extreme<MO>, dim3(blocks), dim3(256), 0, s, F, P.list, P.ctrl); \
        break;
    switch (m) {
        NSGA3_EXT_CASE(2) NSGA3_EXT_CASE(3) NSGA3_EXT_CASE(4) NSGA3_EXT_CASE(5)
        NSGA3_EXT_CASE(6) NSGA3_EXT_CASE(7) NSGA3_EXT_CASE(8) NSGA3_EXT_CASE(9)
        NSGA3_EXT_CASE(10) NSGA3_EXT_CASE(11) NSGA3_EXT_CASE(12) NSGA3_EXT_CASE(13)
        NSGA3_EXT_CASE(14) NSGA3_EXT_CASE(15) NSGA3_EXT_CASE(16)
        default: return hipErrorInvalidValue;
    }
#undef NSGA3_EXT_CASE
    NSGA3_LAUNCH("norm_solve", k_norm_solve, dim3(1), dim3(64), 0, s, F, M, m, P.ctrl, ideal, intercept,
                       extreme, degenerate);
    NSGA3_LAUNCH("norm_apply", k_norm_apply, dim3(blocks), dim3(256), 0, s, F, P.list, m, Fn, P.ctrl);
    return hipGetLastError();
}

}  // namespace nsga3
