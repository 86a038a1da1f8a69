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
#include "steps.h"

namespace nsga3 {

// wide_only: instances with m <= NARROW_M are left to k_norm_fused.
__global__ __launch_bounds__(256) void k_norm_reduce(BatchView bv, int wide_only) {
    __shared__ unsigned s_lo[4][NSGA3_MAX_OBJECTIVES], s_hi[4][NSGA3_MAX_OBJECTIVES];
    __shared__ int s_cnt[4];
    __shared__ int s_base;
    const Local L = locate(bv.pt_pref, bv.B);
    CInst &I = bv.tab[L.b];
    const int x = L.i, M = I.M, m = I.m;
    if (wide_only && m <= NARROW_M) return;  // block-uniform
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
    for (int k = threadIdx.x; k < m; k += 256) {
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
        norm_solve<MO>(I, ctrl->zmin_enc, ctrl->fmax_enc, ctrl->ext_key, I.F, ctrl->zf, ctrl->recip);
    }
}

// The normalization of a whole selection in one pass over the points (the
// ideal point already came from the preparation kernel, over all points):
// the S_t list, the per-objective maximum over S_t, and the ASF extreme
// search; the association outputs of rows outside S_t are set up on the
// way. Every block of an instance's padded point range takes part, and the
// last to finish solves for the intercepts. Grid: all instances' padded
// points (one launch per m; blocks of other instances leave at once).
template <int MO>
__global__ __launch_bounds__(256) void k_norm_fused(BatchView bv) {
    __shared__ unsigned s_hi[4][MO];
    __shared__ u64 s_key[4][MO];
    __shared__ int s_cnt[4];
    __shared__ int s_base;
    __shared__ int s_last;
    const Local L = locate(bv.pt_pref, bv.B);
    CInst &I = bv.tab[L.b];
    if (I.m != MO) return;  // block-uniform
    const int x = L.i, M = I.M;
    Ctrl *ctrl = I.P.ctrl;
    const int l = I.front_info[0];
    const bool in = x < M && I.rank[x] >= 0 && I.rank[x] <= l;
    if (x < M) {
        if (in) I.P.akey[x] = ~0ull;
        else {
            I.pi[x] = -1;
            I.dist[x] = -1.0f;
        }
    }
    const int lane = lane_id();
    const int wv = threadIdx.x >> 6;
    const u64 bal = ballot(in);
    if (lane == 0) s_cnt[wv] = __popcll(bal);
    float fp[MO], g[MO];
#pragma unroll
    for (int k = 0; k < MO; ++k) {
        const float v = in ? I.F[(size_t)x * MO + k] : 0.0f;
        const unsigned hi = wave_max_u32(in ? f2ord(v) : 0u);
        if (lane == 0) s_hi[wv][k] = hi;
        fp[k] = in ? v - ord2f(ctrl->zmin_enc[k]) : 0.0f;
        g[k] = 1e6f * fp[k];
    }
    // ASF_k = max(f'_k, max_{j != k} 1e6 f'_j): largest and second largest g
    float g1 = g[0], g2 = -INFINITY;
    int p1 = 0;
#pragma unroll
    for (int k = 1; k < MO; ++k) {
        if (g[k] > g1) { g2 = g1; g1 = g[k]; p1 = k; }
        else if (g[k] > g2) g2 = g[k];
    }
#pragma unroll
    for (int k = 0; k < MO; ++k) {
        const float asf = fmaxf(fp[k], k == p1 ? g2 : g1);
        const u64 key = in ? (((u64)__float_as_uint(asf) << 32) | (unsigned)x) : ~0ull;
        const u64 wkey = wave_min_u64(key);
        if (lane == 0) s_key[wv][k] = wkey;
    }
    lds_barrier();
    const int total = uniform(s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3]);
    if (total > 0) {
        if (threadIdx.x == 0) s_base = atomicAdd(&ctrl->list_count, total);
        if ((int)threadIdx.x < MO) {
            const int k = threadIdx.x;
            const unsigned hi = max(max(s_hi[0][k], s_hi[1][k]), max(s_hi[2][k], s_hi[3][k]));
            u64 bkey = s_key[0][k];
#pragma unroll
            for (int v = 1; v < 4; ++v) bkey = s_key[v][k] < bkey ? s_key[v][k] : bkey;
            atomicMax(&ctrl->fmax_enc[k], hi);
            atomicMin(&ctrl->ext_key[k], bkey);
        }
        lds_barrier();
        int off = uniform(s_base);
        for (int v = 0; v < wv; ++v) off += s_cnt[v];
        if (in) I.P.list[off + mbcnt(bal)] = x;
    }
    lds_barrier();  // every atomic of the block is issued
    if (threadIdx.x == 0) {
        // release: this block's maxima and minima are performed before the
        // count; the last block acquires them all
        const int nblk = (bv.pt_pref[L.b + 1] - bv.pt_pref[L.b]) / 256;
        const int done = __hip_atomic_fetch_add(&ctrl->ext_done, 1, __ATOMIC_ACQ_REL,
                                                __HIP_MEMORY_SCOPE_AGENT);
        s_last = done == nblk - 1;
    }
    lds_barrier();
    if (s_last && threadIdx.x < 64) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        norm_solve<MO>(I, ctrl->zmin_enc, ctrl->fmax_enc, ctrl->ext_key, I.F, ctrl->zf, ctrl->recip);
    }
}

// ASF extreme search for m > NARROW_M, over the S_t list (the ideal point is
// final): per point the two largest of 1e6 f'_j, then per axis k the key
// (ASF_k bits, index) min-reduced per wave and block, one atomic per block
// and axis. The same float operations as k_norm_extreme. Grid: padded points
// of all instances; blocks of other instances, or past the list, leave.
__global__ __launch_bounds__(256) void k_norm_extreme_wide(BatchView bv) {
    __shared__ u64 s_key[4][NSGA3_MAX_OBJECTIVES];
    const Local L = locate(bv.pt_pref, bv.B);
    CInst &I = bv.tab[L.b];
    const int m = I.m;
    if (m <= NARROW_M) return;  // block-uniform
    Ctrl *ctrl = I.P.ctrl;
    const int n = ctrl->list_count;
    const int base = L.i - (int)threadIdx.x;
    if (base >= n) return;  // block-uniform
    const int i = L.i;
    const bool in = i < n;
    const int x = in ? I.P.list[i] : 0;
    const float *f = I.F + (size_t)x * m;
    float g1 = -INFINITY, g2 = -INFINITY;
    int p1 = 0;
    for (int k = 0; k < m; ++k) {
        const float g = 1e6f * (in ? f[k] - ord2f(ctrl->zmin_enc[k]) : 0.0f);
        if (k == 0 || g > g1) {
            if (k > 0) g2 = g1;
            g1 = g;
            p1 = k;
        } else if (g > g2) {
            g2 = g;
        }
    }
    const int wv = threadIdx.x >> 6;
    for (int k = 0; k < m; ++k) {
        const float fp = in ? f[k] - ord2f(ctrl->zmin_enc[k]) : 0.0f;
        const float asf = fmaxf(fp, k == p1 ? g2 : g1);
        const u64 key = in ? (((u64)__float_as_uint(asf) << 32) | (unsigned)x) : ~0ull;
        const u64 wkey = wave_min_u64(key);
        if (lane_id() == 0) s_key[wv][k] = wkey;
    }
    lds_barrier();
    for (int k = threadIdx.x; k < m; k += 256) {
        u64 bkey = s_key[0][k];
#pragma unroll
        for (int v = 1; v < 4; ++v) bkey = s_key[v][k] < bkey ? s_key[v][k] : bkey;
        if (bkey != ~0ull) atomicMin(&ctrl->ext_key[k], bkey);
    }
}

// Intercepts for m > NARROW_M: one workgroup per instance (others leave).
// The same elimination as norm_solve (largest |pivot|, least position on
// ties; every product and difference rounded separately), on the m x m
// matrix in the workspace: rows stay in place and a permutation holds their
// positions, and each column's updates are spread over the workgroup. Back
// substitution goes column by column (updates of the right-hand side in
// parallel), so its sums run in another order than a row-by-row
// substitution: the intercepts agree with one to rounding, not bit for bit.
constexpr int SOLVE_THREADS = 1024;

__global__ __launch_bounds__(SOLVE_THREADS) void k_norm_solve_wide(BatchView bv) {
    CInst &I = bv.tab[blockIdx.x];
    const int m = I.m;
    if (m <= NARROW_M) return;
    __shared__ double s_val[SOLVE_THREADS / 64];
    __shared__ int s_pos[SOLVE_THREADS / 64];
    __shared__ double s_f[NSGA3_MAX_OBJECTIVES];
    __shared__ int s_perm[NSGA3_MAX_OBJECTIVES];
    __shared__ int s_flag[2];
    __shared__ double s_b;
    Ctrl *ctrl = I.P.ctrl;
    double *E = I.P.emat;                 // [m][m], row-major, physical rows
    double *rhs = E + (size_t)m * m;      // [m]
    double *colmax = rhs + m;             // [m]
    double *bsol = colmax + m;            // [m]
    const int tid = threadIdx.x, M = I.M;
    const int lane = lane_id(), wv = tid >> 6;
    if (tid == 0) { s_flag[0] = 0; s_flag[1] = 0; }
    lds_barrier();
    for (int k = tid; k < m; k += SOLVE_THREADS) {
        const float zf = ord2f(ctrl->zmin_enc[k]);
        int ek = (int)(unsigned)(ctrl->ext_key[k] & 0xffffffffull);
        if (ek < 0 || ek >= M) { ek = 0; atomicOr(&s_flag[0], 1); }
        ctrl->zf[k] = zf;
        I.ideal[k] = zf;
        I.extreme[k] = ek;
        s_perm[k] = k;
        rhs[k] = 1.0;
    }
    __syncthreads();
    const int bad = uniform(s_flag[0]);
    if (bad && tid == 0) atomicOr(&ctrl->status, ST_INTERNAL);
    // E[i][j] = f(e_i)_j - z_j in FP64
    for (int i = wv; i < m; i += SOLVE_THREADS / 64) {
        const int ei = I.extreme[i];
        for (int j = lane; j < m; j += 64)
            E[(size_t)i * m + j] = (double)I.F[(size_t)ei * m + j] - (double)ctrl->zf[j];
    }
    __syncthreads();
    for (int j = tid; j < m; j += SOLVE_THREADS) {
        double cm = 0.0;
        for (int i = 0; i < m; ++i) cm = fmax(cm, fabs(E[(size_t)i * m + j]));
        colmax[j] = cm;
    }
    __syncthreads();
    int degen = bad;
    for (int c = 0; c < m && !degen; ++c) {
        // pivot: largest |E| in column c over positions >= c, least position on ties
        double bv_ = -1.0;
        int bp = 0x7fffffff;
        for (int p = c + tid; p < m; p += SOLVE_THREADS) {
            const double v = fabs(E[(size_t)s_perm[p] * m + c]);
            if (v > bv_) { bv_ = v; bp = p; }
        }
        // wave, then workgroup argmax (ties to the least position)
        for (int o = 32; o > 0; o >>= 1) {
            const double ov = __shfl_xor(bv_, o, 64);
            const int op = __shfl_xor(bp, o, 64);
            if (ov > bv_ || (ov == bv_ && op < bp)) { bv_ = ov; bp = op; }
        }
        if (lane == 0) { s_val[wv] = bv_; s_pos[wv] = bp; }
        __syncthreads();
        if (tid == 0) {
            double v = s_val[0];
            int p = s_pos[0];
            for (int w = 1; w < SOLVE_THREADS / 64; ++w)
                if (s_val[w] > v || (s_val[w] == v && s_pos[w] < p)) { v = s_val[w]; p = s_pos[w]; }
            const double cmx = colmax[c];
            if (cmx == 0.0 || v < 1e-10 * cmx) {
                s_flag[1] = 1;
            } else if (p != c) {
                const int t = s_perm[c];
                s_perm[c] = s_perm[p];
                s_perm[p] = t;
            }
        }
        __syncthreads();
        if (uniform(s_flag[1])) { degen = 1; break; }
        const int rc = s_perm[c];
        const double acc = E[(size_t)rc * m + c];
        const double rr = rhs[rc];
        for (int p = c + 1 + tid; p < m; p += SOLVE_THREADS) {
            const int r = s_perm[p];
            const double f = E[(size_t)r * m + c] / acc;
            s_f[p] = f;
            rhs[r] = __dsub_rn(rhs[r], __dmul_rn(f, rr));
        }
        __syncthreads();
        // columns c+1 .. m-1 of the rows at positions c+1 .. m-1: a wave per
        // row, lanes along it
        for (int p = c + 1 + wv; p < m; p += SOLVE_THREADS / 64) {
            const int r = s_perm[p];
            const double f = s_f[p];
            for (int j = c + 1 + lane; j < m; j += 64)
                E[(size_t)r * m + j] = __dsub_rn(E[(size_t)r * m + j], __dmul_rn(f, E[(size_t)rc * m + j]));
        }
        __syncthreads();
    }
    if (!degen) {
        for (int i = m - 1; i >= 0; --i) {
            if (tid == 0) {
                const int r = s_perm[i];
                s_b = rhs[r] / E[(size_t)r * m + i];
                bsol[i] = s_b;
            }
            __syncthreads();
            const double bi = s_b;
            for (int p = tid; p < i; p += SOLVE_THREADS) {
                const int r = s_perm[p];
                rhs[r] = __dsub_rn(rhs[r], __dmul_rn(E[(size_t)r * m + i], bi));
            }
            __syncthreads();
        }
        for (int k = tid; k < m; k += SOLVE_THREADS) {
            const double bk = bsol[k];
            const double fk = (double)ord2f(ctrl->fmax_enc[k]) - (double)ctrl->zf[k];
            const double a = 1.0 / bk;
            if (!(bk > 0.0) || !isfinite(a) || a < 1e-6 * fk) atomicOr(&s_flag[1], 1);
        }
        __syncthreads();
        degen = uniform(s_flag[1]);
    }
    for (int k = tid; k < m; k += SOLVE_THREADS) {
        const double fk = (double)ord2f(ctrl->fmax_enc[k]) - (double)ctrl->zf[k];
        const double ak = degen ? (fk > 0.0 ? fk : 1.0) : 1.0 / bsol[k];
        I.intercept[k] = ak;
        ctrl->recip[k] = (float)(1.0 / ak);
    }
    if (tid == 0) *I.degenerate = degen;
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

// The one-pass normalization of group g (m <= NARROW_M) of a whole selection.
void launch_norm_fused_group(const HostPlan &hp, const BatchView &bv, int g, hipStream_t s) {
    const unsigned pblocks = (unsigned)(hp.npt / 256);
#define NSGA3_FUSED_CASE(MO)                                                                   \
    case MO:                                                                                   \
        NSGA3_LAUNCH("norm_fused", k_norm_fused<MO>, dim3(pblocks), dim3(256), 0, s, bv);      \
        break;
    switch (hp.grp_m[g]) {
        NSGA3_FUSED_CASE(2) NSGA3_FUSED_CASE(3) NSGA3_FUSED_CASE(4) NSGA3_FUSED_CASE(5)
        NSGA3_FUSED_CASE(6) NSGA3_FUSED_CASE(7) NSGA3_FUSED_CASE(8) NSGA3_FUSED_CASE(9)
        NSGA3_FUSED_CASE(10) NSGA3_FUSED_CASE(11) NSGA3_FUSED_CASE(12)
        NSGA3_FUSED_CASE(13) NSGA3_FUSED_CASE(14) NSGA3_FUSED_CASE(15)
        NSGA3_FUSED_CASE(16)
        default: break;  // m > NARROW_M: launch_normalize's general kernels
    }
#undef NSGA3_FUSED_CASE
}

hipError_t launch_normalize(const HostPlan &hp, const BatchView &bv, hipStream_t s) {
    const unsigned pblocks = (unsigned)(hp.npt / 256);
    bool wide = false;
    for (int g = 0; g < hp.ngroups; ++g) wide |= hp.grp_m[g] > NARROW_M;
    const bool select = (bv.run & RUN_ND) && (bv.run & RUN_ASSOC);
    if (select) {
        // a whole selection: one pass for m <= NARROW_M (the ideal point came
        // with the preparation), Fn formed inside the association sweep
        for (int g = 0; g < hp.ngroups; ++g) launch_norm_fused_group(hp, bv, g, s);
        if (!wide) return hipGetLastError();
    }
    // list, ideal point and maxima over S_t (for m > NARROW_M only, in a
    // whole selection), then the extreme search per m
    NSGA3_LAUNCH("norm_reduce", k_norm_reduce, dim3(pblocks), dim3(256), 0, s, bv, select ? 1 : 0);
    for (int g = 0; g < hp.ngroups; ++g) {
#define NSGA3_EXT_CASE(MO)                                                                     \
    case MO:                                                                                   \
        if (!select)                                                                           \
            NSGA3_LAUNCH("norm_extreme", k_norm_extreme<MO>, dim3(pblocks), dim3(256), 0, s,   \
                         bv, hp.grp_start[g], hp.grp_start[g + 1] - hp.grp_start[g], 0);       \
        break;
        switch (hp.grp_m[g]) {
            NSGA3_EXT_CASE(2) NSGA3_EXT_CASE(3) NSGA3_EXT_CASE(4) NSGA3_EXT_CASE(5)
            NSGA3_EXT_CASE(6) NSGA3_EXT_CASE(7) NSGA3_EXT_CASE(8) NSGA3_EXT_CASE(9)
            NSGA3_EXT_CASE(10) NSGA3_EXT_CASE(11) NSGA3_EXT_CASE(12) NSGA3_EXT_CASE(13)
            NSGA3_EXT_CASE(14) NSGA3_EXT_CASE(15) NSGA3_EXT_CASE(16)
            default: break;
        }
#undef NSGA3_EXT_CASE
    }
    if (wide) {
        NSGA3_LAUNCH("norm_extreme", k_norm_extreme_wide, dim3(pblocks), dim3(256), 0, s, bv);
        NSGA3_LAUNCH("norm_solve", k_norm_solve_wide, dim3(hp.B), dim3(SOLVE_THREADS), 0, s, bv);
    }
    // a whole selection forms Fn inside the association sweep instead
    if (!(bv.run & RUN_ASSOC))
        NSGA3_LAUNCH("norm_apply", k_norm_apply, dim3(pblocks), dim3(256), 0, s, bv);
    return hipGetLastError();
}

}  // namespace nsga3
