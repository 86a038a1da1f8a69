// Association (paper Sec. II-C: each solution goes to the reference point of
// least perpendicular distance; Eq. 1, read as ||f|| sin(theta), the true
// perpendicular distance; Algorithm 2: argmin and min over the reference axis),
// for a batch of independent instances.
//
// The distance tensor of the paper (2N x H) is never materialized: a wave
// holds 64 points of S_t in its lanes and sweeps a slice of the unit
// reference directions, read through the scalar cache from a
// structure-of-arrays copy. The distance is formed from the explicit
// residual r = f - (f . w) w, whose FP32 rounding error scales with ||f||
// rather than with the (possibly tiny) distance. References go in groups of
// eight reduced by min alone (one compare with the running best per group;
// the index is recovered once per slice), and up to four objectives the
// next group's directions load while the current group is computed. Slices
// are merged with a 64-bit atomic min on (d^2 bits << 32 | j): least
// distance, then least j.
//
// Kernels:
//   k_assoc_list   (stage call) S_t list, key init, pi = dist = -1 outside S_t
//   k_associate    the fused sweep; slices merge by a 64-bit atomic min
//   k_assoc_final  pi and dist from the merged keys; in a whole selection
//                  also the niche counts rho (fronts < l) and c (front l)
#include <utility>

#include "steps.h"

namespace nsga3 {

__global__ __launch_bounds__(256) void k_assoc_list(BatchView bv) {
    const Local L = locate(bv.pt_pref, bv.B);
    CInst &I = bv.tab[L.b];
    const int t = L.i;
    const int l = I.front_info[0];
    const bool in = t < I.M && I.rank[t] >= 0 && I.rank[t] <= l;
    if (t < I.M && !in) {
        I.pi[t] = -1;
        I.dist[t] = -1.0f;
    }
    const u64 bal = ballot(in);
    if (bal == 0) return;
    int base = 0;
    if (lane_id() == 0) base = atomicAdd(&I.P.ctrl->list_count, __popcll(bal));
    base = __shfl(base, 0, 64);
    if (in) {
        I.P.list[base + mbcnt(bal)] = t;
        I.P.akey[t] = ~0ull;
    }
}

// Merges a wave's best (d^2, reference) of its slice into the keys of its
// 64 list entries: least distance, then least reference index. A fence per
// wave to let the last slice read the merged keys would write back the L2
// cache of the wave's XCD every time; the keys are read by k_assoc_final,
// after the launch boundary, instead.
__device__ __forceinline__ void assoc_merge(CInst &I, int x, bool in, bool any, float best,
                                            int bj) {
    if (in && any) {
        const u64 key = ((u64)__float_as_uint(best) << 32) | (unsigned)bj;
        atomicMin(&I.P.akey[x], key);
    }
}

// pi and dist from the merged keys; in a whole selection also the niche
// counts rho (fronts < l) and c (front l). Grid: padded points of all
// instances (list positions).
__global__ __launch_bounds__(256) void k_assoc_final(BatchView bv) {
    const Local L = locate(bv.pt_pref, bv.B);
    CInst &I = bv.tab[L.b];
    const int n = I.P.ctrl->list_count;
    if (L.i >= n) return;
    const int x = I.P.list[L.i];
    const u64 key = I.P.akey[x];
    int jm = (int)(unsigned)(key & 0xffffffffull);
    if (jm < 0 || jm >= I.H) {
        atomicOr(&I.P.ctrl->status, ST_INTERNAL);
        jm = 0;
    }
    I.pi[x] = jm;
    I.dist[x] = sqrtf(__uint_as_float((unsigned)(key >> 32)));
    if (bv.run & RUN_NICHE) {
        const int l = I.front_info[0];
        atomicAdd(I.rank[x] < l ? &I.P.rho[jm] : &I.P.cnt[jm], 1);
    }
}

// References are swept in groups of ASSOC_G: a group's distances are reduced
// by min alone, and only the group's least distance is compared with the
// running best (strictly less, so the first group that reaches the final
// least distance is the one kept). The reference index is then found once:
// the first j of the kept group whose recomputed distance equals the best,
// which is the least j at the least distance, as a reference-by-reference
// strict compare would keep.
constexpr int ASSOC_G = 8;

// Blocks of ASSOC_BLK references, unrolled, load the directions of the next
// group through the scalar cache while the current group is computed (two
// groups of MO x ASSOC_G directions in scalar registers: up to
// ASSOC_BLK_MAX_M objectives).
constexpr int ASSOC_BLK = 64;
constexpr int ASSOC_BLK_MAX_M = 4;

template <int MO>
struct AssocW {
    float w[MO][ASSOC_G];
};

template <int MO>
__device__ __forceinline__ void assoc_load(const NSGA3_RO float *wn, int Hp, int j,
                                           AssocW<MO> &g) {
#pragma unroll
    for (int k = 0; k < MO; ++k)
#pragma unroll
        for (int r = 0; r < ASSOC_G; ++r) g.w[k][r] = wn[(size_t)k * Hp + j + r];
}

// Group g of a block: scalar loads return in any order, so a wait for the
// current group would also wait for loads issued after it; the group waits
// first, then issues the next group's loads, then computes.
template <int MO, int g>
__device__ __forceinline__ void assoc_block_group(const float (&f)[MO], const NSGA3_RO float *wn,
                                                  int Hp, int j, AssocW<MO> &cur, AssocW<MO> &nxt,
                                                  float &best, int &bg) {
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (g + 1 < ASSOC_BLK / ASSOC_G) assoc_load<MO>(wn, Hp, j + (g + 1) * ASSOC_G, nxt);
    __builtin_amdgcn_sched_barrier(0);
    float gm = INFINITY;
#pragma unroll
    for (int r = 0; r < ASSOC_G; ++r) {
        float w[MO];
#pragma unroll
        for (int k = 0; k < MO; ++k) w[k] = cur.w[k][r];
        const float d2 = assoc_d2<MO>(f, (const float *)w, 1, 0);
        gm = r == 0 ? d2 : fminf(gm, d2);
    }
    if (gm < best) { best = gm; bg = j + g * ASSOC_G; }
    cur = nxt;
}

template <int MO, int... Gs>
__device__ __forceinline__ void assoc_block(std::integer_sequence<int, Gs...>, const float (&f)[MO],
                                            const NSGA3_RO float *wn, int Hp, int j, float &best,
                                            int &bg) {
    AssocW<MO> cur, nxt;
    assoc_load<MO>(wn, Hp, j, cur);
    (assoc_block_group<MO, Gs>(f, wn, Hp, j, cur, nxt, best, bg), ...);
}

// Work item = (block of 64 list entries, slice of R references) of one
// instance of the m-group order[gs .. gs + gn). Items cover the largest
// possible S_t; items past the actual list length exit at once. The item is
// wave-uniform, so the unit directions come through the scalar cache.
template <int MO>
__global__ __launch_bounds__(256) void k_associate(BatchView bv, int gs, int gn, long long item0,
                                                    long long n_items) {
    const long long gitem = uniform(item0 + (long long)blockIdx.x * 4 + (threadIdx.x >> 6));
    if (gitem >= item0 + n_items) return;
    const int gi = uniform(find_range(bv.asc_pref + gs, gn, gitem));
    CInst &I = bv.tab[bv.order[gs + gi]];
    const long long item = gitem - bv.asc_pref[gs + gi];
    const int n = I.P.ctrl->list_count;
    const int pb = (int)(item / I.nslice);
    const int sl = (int)(item % I.nslice);
    if (pb * 64 >= n) return;
    const int i = pb * 64 + lane_id();
    const bool in = i < n;
    const int x = in ? I.P.list[i] : I.P.list[pb * 64];
    // in a whole selection Fn is formed here from F, the ideal point and the
    // intercepts (the same float32 operations as the normalization's output)
    const bool fused = (bv.run & RUN_NORM) != 0;
    const float *__restrict__ Fn = fused ? I.F : I.Fn;
    // unit directions: written by k_prep, read-only here (invariant loads)
    const NSGA3_RO float *wn = (const NSGA3_RO float *)I.P.wn;
    const int H = I.H, Hp = I.Hp;
    // ideal point and reciprocal intercepts: written by the normalization,
    // read-only here (invariant loads)
    const NSGA3_RO Ctrl *cc = (const NSGA3_RO Ctrl *)I.P.ctrl;
    float f[MO];
#pragma unroll
    for (int k = 0; k < MO; ++k) {
        f[k] = Fn[(size_t)x * MO + k];
        if (fused) f[k] = (f[k] - cc->zf[k]) * cc->recip[k];
    }
    const int h0 = sl * I.R;
    const int h1 = min(h0 + I.R, H);
    float best = INFINITY;
    int bg = h0;  // first reference of the kept group (or kept tail reference)
    int j = h0;
    if constexpr (MO <= ASSOC_BLK_MAX_M)
        for (; j + ASSOC_BLK <= h1; j += ASSOC_BLK)
            assoc_block<MO>(std::make_integer_sequence<int, ASSOC_BLK / ASSOC_G>{}, f, wn, Hp, j,
                            best, bg);
    for (; j + ASSOC_G <= h1; j += ASSOC_G) {
        float gm = assoc_d2<MO>(f, wn, Hp, j);
#pragma unroll
        for (int r = 1; r < ASSOC_G; ++r) gm = fminf(gm, assoc_d2<MO>(f, wn, Hp, j + r));
        if (gm < best) { best = gm; bg = j; }
    }
    for (; j < h1; ++j) {
        const float d2 = assoc_d2<MO>(f, wn, Hp, j);
        if (d2 < best) { best = d2; bg = j; }
    }
    // the kept group holds a distance equal to best at or after bg (a tail
    // reference is its own first match); nothing below infinity keeps h0
    int bj = bg;
    if (best < INFINITY) {
        const int ge = min(bg + ASSOC_G, h1);
        for (int jj = ge - 1; jj >= bg; --jj)
            if (assoc_d2<MO>(f, wn, Hp, jj) == best) bj = jj;
    }
    assoc_merge(I, x, in, h0 < h1, best, bj);
}

// Association for m > NARROW_M: the same work items (64 list entries in the
// lanes, a slice of references), with a point's objectives streamed in
// chunks of AW_KC. References go in groups of AW_RG: one pass over the chunks
// forms every projection p_j = f . w_j of the group, a second the squared
// residuals sum_k (f_k - p_j w_jk)^2 (each sum by chunks, then over chunks).
// Unit directions are rows (wn[j][k]), read through the scalar cache.
constexpr int AW_KC = 16;
constexpr int AW_RG = 32;

__global__ __launch_bounds__(256) void k_associate_wide(BatchView bv, int gs, int gn,
                                                         long long item0, long long n_items) {
    const long long gitem = uniform(item0 + (long long)blockIdx.x * 4 + (threadIdx.x >> 6));
    if (gitem >= item0 + n_items) return;
    const int gi = uniform(find_range(bv.asc_pref + gs, gn, gitem));
    CInst &I = bv.tab[bv.order[gs + gi]];
    const long long item = gitem - bv.asc_pref[gs + gi];
    const int n = I.P.ctrl->list_count;
    const int pb = (int)(item / I.nslice);
    const int sl = (int)(item % I.nslice);
    if (pb * 64 >= n) return;
    const int i = pb * 64 + lane_id();
    const bool in = i < n;
    const int x = in ? I.P.list[i] : I.P.list[pb * 64];
    const bool fused = (bv.run & RUN_NORM) != 0;
    const float *__restrict__ src = (fused ? I.F : I.Fn) + (size_t)x * I.m;
    const NSGA3_RO float *wn = (const NSGA3_RO float *)I.P.wn;
    const NSGA3_RO Ctrl *cc = (const NSGA3_RO Ctrl *)I.P.ctrl;
    const int H = I.H, m = I.m;
    const int h0 = sl * I.R;
    const int h1 = min(h0 + I.R, H);
    float best = INFINITY;
    int bj = h0;
    auto load_f = [&](int k0, float (&f)[AW_KC]) {
#pragma unroll
        for (int kk = 0; kk < AW_KC; ++kk) {
            const int k = k0 + kk;
            float v = 0.0f;
            if (k < m) {
                v = src[k];
                if (fused) v = (v - cc->zf[k]) * cc->recip[k];
            }
            f[kk] = v;
        }
    };
    for (int g0 = h0; g0 < h1; g0 += AW_RG) {
        const int ng = min(AW_RG, h1 - g0);
        float p[AW_RG], d2[AW_RG];
#pragma unroll
        for (int r = 0; r < AW_RG; ++r) p[r] = d2[r] = 0.0f;
        for (int k0 = 0; k0 < m; k0 += AW_KC) {
            float f[AW_KC];
            load_f(k0, f);
#pragma unroll
            for (int r = 0; r < AW_RG; ++r) {
                if (r >= ng) break;
                const NSGA3_RO float *w = wn + (size_t)(g0 + r) * m + k0;
                float acc = 0.0f;
#pragma unroll
                for (int kk = 0; kk < AW_KC; ++kk)
                    if (k0 + kk < m) acc = fmaf(f[kk], w[kk], acc);
                p[r] += acc;
            }
        }
        for (int k0 = 0; k0 < m; k0 += AW_KC) {
            float f[AW_KC];
            load_f(k0, f);
#pragma unroll
            for (int r = 0; r < AW_RG; ++r) {
                if (r >= ng) break;
                const NSGA3_RO float *w = wn + (size_t)(g0 + r) * m + k0;
                float acc = 0.0f;
#pragma unroll
                for (int kk = 0; kk < AW_KC; ++kk) {
                    if (k0 + kk < m) {
                        const float rr = fmaf(-p[r], w[kk], f[kk]);
                        acc = fmaf(rr, rr, acc);
                    }
                }
                d2[r] += acc;
            }
        }
#pragma unroll
        for (int r = 0; r < AW_RG; ++r)
            if (r < ng && d2[r] < best) { best = d2[r]; bj = g0 + r; }
    }
    assoc_merge(I, x, in, h0 < h1, best, bj);
}

// The association sweep of group g (instances of one m).
void launch_associate_group(const HostPlan &hp, const BatchView &bv, int g, hipStream_t s) {
    const int gs = hp.grp_start[g], gn = hp.grp_start[g + 1] - gs;
    const long long item0 = hp.grp_asc[g], n_items = hp.grp_asc[g + 1] - item0;
    const unsigned blocks = (unsigned)((n_items + 3) / 4);
#define NSGA3_ASSOC_CASE(MO)                                                                   \
    case MO:                                                                                   \
        NSGA3_LAUNCH("associate", k_associate<MO>, dim3(blocks), dim3(256), 0, s, bv, gs, gn,  \
                     item0, n_items);                                                          \
        break;
    switch (hp.grp_m[g]) {
        NSGA3_ASSOC_CASE(2) NSGA3_ASSOC_CASE(3) NSGA3_ASSOC_CASE(4) NSGA3_ASSOC_CASE(5)
        NSGA3_ASSOC_CASE(6) NSGA3_ASSOC_CASE(7) NSGA3_ASSOC_CASE(8) NSGA3_ASSOC_CASE(9)
        NSGA3_ASSOC_CASE(10) NSGA3_ASSOC_CASE(11) NSGA3_ASSOC_CASE(12) NSGA3_ASSOC_CASE(13)
        NSGA3_ASSOC_CASE(14) NSGA3_ASSOC_CASE(15) NSGA3_ASSOC_CASE(16)
        default:
            NSGA3_LAUNCH("associate", k_associate_wide, dim3(blocks), dim3(256), 0, s, bv, gs, gn,
                         item0, n_items);
            break;
    }
#undef NSGA3_ASSOC_CASE
}

hipError_t launch_associate(const HostPlan &hp, const BatchView &bv, hipStream_t s,
                            bool sweeps_done) {
    const unsigned pblocks = (unsigned)(hp.npt / 256);
    if (!sweeps_done) {
        if (!(bv.run & RUN_NORM))
            NSGA3_LAUNCH("assoc_list", k_assoc_list, dim3(pblocks), dim3(256), 0, s, bv);
        for (int g = 0; g < hp.ngroups; ++g) launch_associate_group(hp, bv, g, s);
    }
    NSGA3_LAUNCH("assoc_final", k_assoc_final, dim3(pblocks), dim3(256), 0, s, bv);
    return hipGetLastError();
}

}  // namespace nsga3
