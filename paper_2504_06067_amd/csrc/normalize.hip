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
//   k_norm_extreme  per-axis ASF argmin over S_t as a 64-bit (value, index) min;
//                   the last block of an instance then solves for the
//                   intercepts with one wave (FP64 elimination, degeneracy
//                   tests)
//   k_norm_apply    Fn = (f - z) * (1 / a) over S_t (stage call; a whole
//                   selection forms Fn in the association sweep)
#include "nsga3_internal.h"

namespace nsga3 {

__global__ __launch_bounds__(256) void k_norm_reduce(BatchView bv) {
    __shared__ unsigned s_lo[4][NSGA3_MAX_OBJECTIVES], s_hi[4][NSGA3_MAX_OBJECTIVES];
    __shared__ int s_cnt[4];
    __shared__ int s_base;
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
    // per-wave, then per-block reductions: one atomic per block and quantity
    const int lane = lane_id();
    const int wv = threadIdx.x >> 6;
    const u64 bal = ballot(in);
    if (lane == 0) s_cnt[wv] = __popcll(bal);
    for (int k = 0; k < m; ++k) {
        const float v = in ? I.F[(size_t)x * m + k] : 0.0f;
        const unsigned lo = wave_min_u32(in ? f2ord(v) : 0xffffffffu);
        const unsigned hi = wave_max_u32(in ? f2ord(v) : 0u);
        if (lane == 0) {
            s_lo[wv][k] = lo;
            s_hi[wv][k] = hi;
        }
    }
    lds_barrier();
    const int total = uniform(s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3]);
    if (total == 0) return;  // block-uniform
    if (threadIdx.x == 0) s_base = atomicAdd(&ctrl->list_count, total);
    if ((int)threadIdx.x < m) {
        const int k = threadIdx.x;
        const unsigned lo = min(min(s_lo[0][k], s_lo[1][k]), min(s_lo[2][k], s_lo[3][k]));
        const unsigned hi = max(max(s_hi[0][k], s_hi[1][k]), max(s_hi[2][k], s_hi[3][k]));
        atomicMin(&ctrl->zmin_enc[k], lo);
        atomicMax(&ctrl->fmax_enc[k], hi);
    }
    lds_barrier();
    int off = uniform(s_base);
    for (int v = 0; v < wv; ++v) off += s_cnt[v];
    if (in) I.P.list[off + mbcnt(bal)] = x;
}

// Doubles move between lanes as two 32-bit halves.
__device__ __forceinline__ double read_lane_f64(double v, int L) {
    const u64 u = (u64)__double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)u, L);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)(u >> 32), L);
    return __longlong_as_double((long long)(((u64)hi << 32) | lo));
}

// One wave per instance. E[k][j] =
// f(e_k)_j - z_j in FP64; E b = 1 is solved by Gaussian elimination with
// partial pivoting (largest |pivot|, least row on ties), the rows spread over
// the lanes (each row stays in its lane and carries its position; a swap
// exchanges two positions), every product and difference rounded separately;
// a_k = 1 / b_k
// unless degenerate.
template <int MO>
__device__ void norm_solve(CInst &I) {
    Ctrl *ctrl = I.P.ctrl;
    const int lane = lane_id();
    const int M = I.M;
    // ideal point, extreme indices, per-objective span (lane k: objective k)
    int bad = 0;
    double zk = 0.0, fmxk = 0.0;
    int ek = 0;
    if (lane < MO) {
        const float zf = ord2f(ctrl->zmin_enc[lane]);
        zk = (double)zf;
        fmxk = (double)ord2f(ctrl->fmax_enc[lane]) - zk;
        ek = (int)(unsigned)(ctrl->ext_key[lane] & 0xffffffffull);
        if (ek < 0 || ek >= M) { ek = 0; bad = 1; }
        ctrl->zf[lane] = zf;
        I.ideal[lane] = zf;
        I.extreme[lane] = ek;
    }
    int degen = uniform((int)(ballot(bad != 0) != 0));
    if (degen && lane == 0) atomicOr(&ctrl->status, ST_INTERNAL);
    // row i of E in lane i: A[j] = f(e_i)_j - z_j, right-hand side 1
    double A[MO];
    double rhs = 1.0;
#pragma unroll
    for (int j = 0; j < MO; ++j) {
        const double zj = read_lane_f64(zk, j);
        A[j] = lane < MO ? (double)I.F[(size_t)ek * MO + j] - zj : 0.0;
    }
    // largest |entry| per column of the original matrix
    double colmax[MO];
#pragma unroll
    for (int j = 0; j < MO; ++j) {
        const u64 key = lane < MO ? (u64)__double_as_longlong(fabs(A[j])) : 0ull;
        colmax[j] = __longlong_as_double((long long)wave_max_u64(key));
    }
    // Rows stay in their lanes; pos is the row's position in the eliminated
    // matrix (a swap of two positions exchanges two lanes' pos values).
    int pos = lane;
#pragma unroll
    for (int c = 0; c < MO; ++c) {
        if (degen) break;
        // pivot: largest |A[i][c]| over positions i >= c, least position on ties
        const bool cand = lane < MO && pos >= c;
        const u64 key = cand ? (u64)__double_as_longlong(fabs(A[c])) : 0ull;
        const u64 best = wave_max_u64(key);
        const int piv = (int)wave_min_u32(cand && key == best ? (unsigned)pos : 0xffffffffu);
        const double pv = __longlong_as_double((long long)best);
        if (colmax[c] == 0.0 || pv < 1e-10 * colmax[c]) {
            degen = 1;
            break;
        }
        const int lp = __ffsll((long long)ballot(lane < MO && pos == piv)) - 1;  // pivot row's lane
        const int lc = __ffsll((long long)ballot(lane < MO && pos == c)) - 1;    // position c's lane
        if (piv != c) {
            if (lane == lp) pos = c;
            else if (lane == lc) pos = piv;
        }
        const double acc = read_lane_f64(A[c], lp);
        const double rc = read_lane_f64(rhs, lp);
        const bool below = lane < MO && pos > c;
        const double f = below ? A[c] / acc : 0.0;
#pragma unroll
        for (int j = c; j < MO; ++j) {
            const double acj = read_lane_f64(A[j], lp);
            if (below) A[j] = __dsub_rn(A[j], __dmul_rn(f, acj));
        }
        if (below) rhs = __dsub_rn(rhs, __dmul_rn(f, rc));
    }
    double b[MO];
    if (!degen) {
#pragma unroll
        for (int i = MO - 1; i >= 0; --i) {
            const int li = __ffsll((long long)ballot(lane < MO && pos == i)) - 1;  // row at position i
            double s = read_lane_f64(rhs, li);
#pragma unroll
            for (int j = i + 1; j < MO; ++j) s = __dsub_rn(s, __dmul_rn(read_lane_f64(A[j], li), b[j]));
            b[i] = s / read_lane_f64(A[i], li);
        }
    }
    // intercepts, or the per-objective maximum when degenerate
    double ak = 1.0;
#pragma unroll
    for (int k = 0; k < MO; ++k) {
        if (degen) break;
        const double fk = read_lane_f64(fmxk, k);
        if (!(b[k] > 0.0)) { degen = 1; break; }
        const double a = 1.0 / b[k];
        if (!isfinite(a) || a < 1e-6 * fk) { degen = 1; break; }
        if (k == lane) ak = a;
    }
    if (degen) ak = fmxk > 0.0 ? fmxk : 1.0;
    if (lane < MO) {
        I.intercept[lane] = ak;
        ctrl->recip[lane] = (float)(1.0 / ak);
    }
    if (lane == 0) *I.degenerate = degen;
}

// ASF_k(x) = max(f'_k, max_{j != k} 1e6 * f'_j) with f' = f - z >= 0 on S_t,
// so the raw float bits order like the values; ties go to the least index.
// The last of an instance's blocks to finish (a counter in its control block)
// then solves for the intercepts with one wave. Grid: padded points of the
// group's instances (one launch per m).
template <int MO>
__global__ __launch_bounds__(256) void k_norm_extreme(BatchView bv, int gs, int gn, int pt0) {
    const int base = uniform(pt0 + (int)(blockIdx.x * blockDim.x));
    const int gi = uniform(find_range(bv.pt_pref, bv.B, base));
    CInst &I = bv.tab[gi];
    Ctrl *ctrl = I.P.ctrl;
    const int n = ctrl->list_count;
    const int i = base - bv.pt_pref[gi] + (int)threadIdx.x;
    // blocks 0 .. nblk - 1 of the instance take part (block 0 also when S_t is empty)
    const int nblk = n > 0 ? (n + 255) / 256 : 1;
    if (base - bv.pt_pref[gi] >= nblk * 256 || I.m != MO) return;
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
    // per wave, then per block: one atomic per block and objective (atomics on
    // one address are performed one after another)
    __shared__ u64 s_key[4][MO];
    const int wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < MO; ++k) {
        const float other = (k == p1) ? g2 : g1;
        const float asf = fmaxf(fp[k], other);
        const u64 key = in ? (((u64)__float_as_uint(asf) << 32) | (unsigned)x) : ~0ull;
        const u64 wkey = wave_min_u64(key);
        if (lane_id() == 0) s_key[wv][k] = wkey;
    }
    lds_barrier();
    if (threadIdx.x < MO) {
        const int k = threadIdx.x;
        u64 bkey = s_key[0][k];
#pragma unroll
        for (int v = 1; v < 4; ++v) bkey = s_key[v][k] < bkey ? s_key[v][k] : bkey;
        if (bkey != ~0ull) atomicMin(&ctrl->ext_key[k], bkey);
    }
    (void)gs;
    (void)gn;
    __shared__ int s_last;
    lds_barrier();  // every minimum of the block is issued
    if (threadIdx.x == 0) {
        // release: this block's minima are performed before the count; the
        // last block acquires them all
        const int done = __hip_atomic_fetch_add(&ctrl->ext_done, 1, __ATOMIC_ACQ_REL,
                                                __HIP_MEMORY_SCOPE_AGENT);
        s_last = done == nblk - 1;
    }
    lds_barrier();
    if (s_last && threadIdx.x < 64) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        norm_solve<MO>(I);
    }
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
    // a whole selection forms Fn inside the association sweep instead
    if (!(bv.run & RUN_ASSOC))
        NSGA3_LAUNCH("norm_apply", k_norm_apply, dim3(pblocks), dim3(256), 0, s, bv);
    return hipGetLastError();
}

}  // namespace nsga3
