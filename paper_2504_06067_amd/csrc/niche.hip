// Niching (Algorithm 1 niche-selection loop; Algorithm 2 nearest selection,
// cache tensor Q, random selection loop and truncation).
//
// The paper removes the serial loop's cost with a cache tensor and a
// batched while-loop. Here the loop is replaced by its closed form. In the
// sequential loop every reference that still has candidates is served once at
// niche count L, in key order, before any is served at L + 1; references
// interact only through the shared budget K. With
//   P(L) = sum_j min(c_j, max(0, L - rho_j))      (picks needed to fill to L)
// the last complete level is L* = max{L : P(L) <= K}; the r = K - P(L*)
// references of T = {j : rho_j <= L* < rho_j + c_j} with least
// key(seed, 1, j, L*) get one more pick. Each reference then makes its own
// picks at its levels rho_j .. rho_j + t_j - 1: the nearest candidate at
// level 0, otherwise candidate (key(seed, 2, j, L) mod remaining) in
// ascending index order. The result equals the one-pick-per-iteration loop.
//
// For a batch of independent instances (counters are zeroed by k_prep).
//
// Kernels:
//   k_niche_count    rho (fronts < l) and c (front l) per reference (stage
//                    call; a whole selection counts in the association)
//   k_niche_plan     one workgroup per instance: CSR offsets, L*, the r-th
//                    least tag-1 key (counted ranks or radix select),
//                    per-reference pick counts t_j
//   k_niche_scatter  members of front l into per-reference segments
//   k_niche_pick     one wave per reference: sort its segment ascending,
//                    then its picks: decoded all at once from their ranks
//                    (8 to 256 picks), else one by one with a remaining-set
//                    bitmask
//   k_compact        ascending output of S and the picks
//   k_ct_offsets, k_ct_loop   the paper's cache-tensor loop (A/B baseline)
#include <limits.h>

#include "steps.h"

namespace nsga3 {

constexpr int PLAN_THREADS = 1024;
constexpr int PLAN_BINS = 4096;         // radix-select bins (12 bits; 256 per wave)

__device__ __forceinline__ u64 read_lane_u64(u64 x, int L) {
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)x, L);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)(x >> 32), L);
    return ((u64)hi << 32) | lo;
}
constexpr int PICK_CAP = 2048;          // segment length kept in LDS by one wave
constexpr int PICK_DECODE_MAX = 256;    // most picks of a reference decoded in parallel
constexpr int PICK_DECODE_MIN = 8;      // fewer picks: the serial chain is shorter

// Stage call only (a whole selection counts in the association's final pass).
__global__ __launch_bounds__(256) void k_niche_count(BatchView bv) {
    const Local L = locate(bv.pt_pref, bv.B);
    CInst &I = bv.tab[L.b];
    const int x = L.i;
    if (x >= I.M) return;
    const int l = I.front_info[0];
    const int r = I.rank[x];
    if (r < 0 || r > l) return;
    const int p = I.pi[x];
    if (p < 0 || p >= I.H) {
        atomicOr(&I.P.ctrl->status, ST_INTERNAL);
        return;
    }
    atomicAdd(r < l ? &I.P.rho[p] : &I.P.cnt[p], 1);
}

__device__ __forceinline__ long long block_sum_ll(long long v, long long *red) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    lds_barrier();
    if (lane_id() == 0) red[w] = v;
    lds_barrier();
    long long s = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
    return uniform(s);
}

// Plan threads own references strided by PLAN_THREADS (thread t: t, t + T,
// t + 2T, ...; coalesced loads and stores), held in registers PLAN_PER rows
// at a time; larger H takes several groups of rows.
constexpr int PLAN_PER = 12;
constexpr int PLAN_WAVES = PLAN_THREADS / 64;
constexpr int PLAN_TCAP = 2048;  // members of T whose keys are gathered in LDS
// Largest |T| whose threshold key is found by counting ranks (|T|^2
// compares, from LDS); larger ones take the radix passes, whose cost is a
// few block barriers whatever |T|.
constexpr int PLAN_COUNT_MAX = 256;

__device__ __forceinline__ long long block_max_ll(long long v, long long *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, (long long)__shfl_xor(v, o, 64));
    lds_barrier();
    if (lane_id() == 0) red[threadIdx.x >> 6] = v;
    lds_barrier();
    long long m = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) m = max(m, red[i]);
    return uniform(m);
}

// One workgroup per instance.
__global__ __launch_bounds__(PLAN_THREADS) void k_niche_plan(BatchView bv) {
    CInst &I = bv.tab[blockIdx.x];
    const int *__restrict__ rho = I.P.rho;
    const int *__restrict__ cnt = I.P.cnt;
    const int H = I.H;
    const u64 seed = I.seed;
    int *off = I.P.off;
    int *tpick = I.P.tpick;
    Ctrl *ctrl = I.P.ctrl;
    __shared__ long long red[PLAN_WAVES];
    __shared__ unsigned hist[PLAN_BINS];
    __shared__ int wtot[PLAN_PER * PLAN_WAVES];
    __shared__ u64 cand[64];
    __shared__ u64 cand_thr[1];
    __shared__ int s_sel[4];
    __shared__ int s_lev[4];  // L*, |T|, P(L*), L* beyond the level window
    __shared__ int wt2[PLAN_WAVES];
    __shared__ int t_ref[PLAN_TCAP];   // listed members of T: reference, niche count, key
    __shared__ int t_rho[PLAN_TCAP];
    __shared__ u64 t_key[PLAN_TCAP];
    const int tid = threadIdx.x;
    const int wv = uniform((int)(threadIdx.x >> 6));
    const int lane = lane_id();
    const int K = uniform(I.front_info[2]);
    // level differences: +1 at rho_j, -1 at rho_j + c_j (levels < PLAN_BINS)
    int *dlev = (int *)hist;
    for (int q = tid; q < PLAN_BINS; q += PLAN_THREADS) dlev[q] = 0;
    if (tid == 0) s_lev[3] = 0;
    lds_barrier();

    // rows of PLAN_THREADS references; groups of PLAN_PER rows
    const int rows = (H + PLAN_THREADS - 1) / PLAN_THREADS;
    const int groups = (rows + PLAN_PER - 1) / PLAN_PER;
    int rc[PLAN_PER], cc[PLAN_PER];
    auto load_group = [&](int g) {
#pragma unroll
        for (int q = 0; q < PLAN_PER; ++q) {
            const int j = (g * PLAN_PER + q) * PLAN_THREADS + tid;
            rc[q] = j < H ? rho[j] : 0;
            cc[q] = j < H ? cnt[j] : 0;
        }
    };
    load_group(0);
    // Loops over the owned references (group 0 stays loaded when it is the
    // only one).
#define PLAN_FOR(BODY)                                                         \
    for (int g = 0; g < groups; ++g) {                                         \
        if (groups > 1) load_group(g);                                         \
        _Pragma("unroll") for (int q = 0; q < PLAN_PER; ++q) {                 \
            const int j = (g * PLAN_PER + q) * PLAN_THREADS + tid;             \
            if (j < H) {                                                       \
                const int cj = cc[q], rj = rc[q];                              \
                BODY                                                           \
            }                                                                  \
        }                                                                      \
    }

    // exclusive scan of c in reference order, group by group: per row a wave
    // scan; wave 0 scans the (row, wave) totals in order
    long long hi_local = 0;
    int carry = 0;
    for (int g = 0; g < groups; ++g) {
        if (groups > 1) load_group(g);
        int incl[PLAN_PER];
#pragma unroll
        for (int q = 0; q < PLAN_PER; ++q) {
            incl[q] = wave_incl_scan(cc[q]);
            if (lane == 63) wtot[q * PLAN_WAVES + wv] = incl[q];
            const int j = (g * PLAN_PER + q) * PLAN_THREADS + tid;
            if (j < H && cc[q] > 0) {
                if (rc[q] < PLAN_BINS) atomicAdd(&dlev[rc[q]], 1);
                if (rc[q] + cc[q] < PLAN_BINS) atomicAdd(&dlev[rc[q] + cc[q]], -1);
            }
        }
        lds_barrier();
        if (wv == 0) {
            // PLAN_PER * PLAN_WAVES entries in (row, wave) order, three per lane
            static_assert(PLAN_PER * PLAN_WAVES == 3 * 64, "three totals per lane");
            const int e0 = 3 * lane;
            const int t0 = wtot[e0], t1 = wtot[e0 + 1], t2 = wtot[e0 + 2];
            const int sum = t0 + t1 + t2;
            const int ex = wave_incl_scan(sum) - sum + carry;
            wtot[e0] = ex;
            wtot[e0 + 1] = ex + t0;
            wtot[e0 + 2] = ex + t0 + t1;
            if (lane == 63) s_sel[0] = ex + sum;
        }
        lds_barrier();
#pragma unroll
        for (int q = 0; q < PLAN_PER; ++q) {
            const int j = (g * PLAN_PER + q) * PLAN_THREADS + tid;
            if (j < H) {
                off[j] = wtot[q * PLAN_WAVES + wv] + incl[q] - cc[q];
                if (cc[q] > 0) hi_local = max(hi_local, (long long)rc[q] + cc[q]);
            }
        }
        carry = uniform(s_sel[0]);
        lds_barrier();  // wtot and s_sel are reused
    }
    if (groups > 1) load_group(0);
    const long long total = carry;
    if (tid == 0) off[H] = carry;

    if (K >= total) {
        // the whole last front is taken
        PLAN_FOR({ (void)rj; tpick[j] = cj; })
        if (wv == 0) {
            ctrl->all_pick = 1;
            ctrl->lstar = -1;
            ctrl->rpick = 0;
            ctrl->fl_total = (int)total;
            if (K > total) atomicOr(&ctrl->status, ST_INTERNAL);
        }
        return;
    }
    // L* = max{L : P(L) <= K}. With a_l = |{j : rho_j <= l < rho_j + c_j}|
    // (the prefix sum of the level differences), P(L) = a_0 + ... + a_{L-1},
    // so P(L* + 1) = P(L*) + a_{L*} > K >= P(L*), and a_{L*} = |T|. Thread t
    // holds levels 4t .. 4t + 3 of the window [0, PLAN_BINS).
    int Ls, tsize_i;
    long long pl;
    {
        int dv[4], av[4], sd = 0, sa = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) { dv[q] = dlev[4 * tid + q]; sd += dv[q]; }
        const int i1 = wave_incl_scan(sd);
        if (lane == 63) red[wv] = i1;
        lds_barrier();
        int run = i1 - sd;
        for (int v = 0; v < wv; ++v) run += (int)red[v];
#pragma unroll
        for (int q = 0; q < 4; ++q) { run += dv[q]; av[q] = run; sa += run; }
        const int i2 = wave_incl_scan(sa);
        if (lane == 63) wt2[wv] = i2;
        lds_barrier();
        int P = i2 - sa;
        for (int v = 0; v < wv; ++v) P += wt2[v];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int L = 4 * tid + q;
            const int Pn = P + av[q];
            if (P <= K && Pn > K) {
                s_lev[0] = L;
                s_lev[1] = av[q];
                s_lev[2] = P;
            }
            if (L == PLAN_BINS - 1 && Pn <= K) s_lev[3] = 1;
            P = Pn;
        }
        lds_barrier();
        Ls = uniform(s_lev[0]);
        tsize_i = uniform(s_lev[1]);
        pl = uniform(s_lev[2]);
    }
    if (uniform(s_lev[3])) {
        // L* lies beyond the window: binary search over P
        long long lo = PLAN_BINS, hi = block_max_ll(hi_local, red);
        while (hi - lo > 1) {
            const long long mid = (lo + hi) >> 1;
            long long p = 0;
            PLAN_FOR({ p += min((long long)cj, max(0ll, mid - rj)); })
            p = block_sum_ll(p, red);
            if (p <= K) lo = mid; else hi = mid;
        }
        Ls = (int)lo;
        long long p2 = 0;
        int tcount = 0;
        PLAN_FOR({
            p2 += min((long long)cj, max(0ll, (long long)Ls - rj));
            tcount += (cj > 0 && rj <= Ls && Ls < rj + cj);
        })
        pl = block_sum_ll(p2, red);
        tsize_i = (int)block_sum_ll((long long)tcount, red);
    }
    const long long tsize = tsize_i;
    const int r = (int)(K - pl);

    // the r least tag-1 keys of T = {j : rho_j <= L* < rho_j + c_j} get one more
    // pick. The r-th least key is found by radix select, 12 bits per pass from
    // the top; as soon as the keys left in the chosen bin are at most 64, one
    // wave ranks them exactly. Keys of distinct references differ (sm64 is a
    // bijection).
    u64 prefix = 0;
    const bool every = r >= tsize;  // r == |T|: every key of T qualifies
    // Up to PLAN_TCAP members of T are gathered into LDS first, so that each
    // key is hashed once, by one thread (a key costs several 64-bit
    // multiplies, and T is a small, scattered subset of the references).
    const bool listed = r > 0 && r < tsize && tsize <= PLAN_TCAP;
    int ntk = 0;
    if (listed) {
        if (tid == 0) s_sel[3] = 0;
        lds_barrier();
        for (int g = 0; g < groups; ++g) {
            if (groups > 1) load_group(g);
#pragma unroll
            for (int q = 0; q < PLAN_PER; ++q) {
                const int j = (g * PLAN_PER + q) * PLAN_THREADS + tid;
                const bool in_t = j < H && cc[q] > 0 && rc[q] <= Ls && Ls < rc[q] + cc[q];
                const u64 bal = ballot(in_t);
                if (bal == 0) continue;  // wave-uniform
                int base = 0;
                if (lane == 0) base = atomicAdd(&s_sel[3], __popcll(bal));
                base = uniform(base);
                if (in_t) {
                    t_ref[base + mbcnt(bal)] = j;
                    t_rho[base + mbcnt(bal)] = rc[q];
                }
            }
        }
        if (groups > 1) load_group(0);
        lds_barrier();
        ntk = uniform(s_sel[3]);
        for (int e = tid; e < ntk; e += PLAN_THREADS)
            t_key[e] = tie_key(seed, 1u, (unsigned)t_ref[e], (unsigned)Ls);
        lds_barrier();
    }
    if (r > 0 && r < tsize) {
        // keys of the owned members of T (group 0 when it is the only one)
        u64 kc[PLAN_PER];
#pragma unroll
        for (int q = 0; q < PLAN_PER; ++q) kc[q] = 0ull;
        if (!listed && groups == 1) {  // uniform: no key hashed when T is listed
#pragma unroll
            for (int q = 0; q < PLAN_PER; ++q) {
                const int j = q * PLAN_THREADS + tid;
                if (j < H && cc[q] > 0 && rc[q] <= Ls && Ls < rc[q] + cc[q])
                    kc[q] = tie_key(seed, 1u, (unsigned)j, (unsigned)Ls);
            }
        }
        // calls BODY with `key` for every key of T owned by this thread
#define PLAN_KEYS(BODY)                                                                       \
    if (listed) {                                                                             \
        for (int e = tid; e < ntk; e += PLAN_THREADS) {                                       \
            const u64 key = t_key[e];                                                         \
            BODY                                                                              \
        }                                                                                     \
    } else if (groups == 1) {                                                                 \
        _Pragma("unroll") for (int q = 0; q < PLAN_PER; ++q) {                                \
            const int j = q * PLAN_THREADS + tid;                                             \
            if (j < H && cc[q] > 0 && rc[q] <= Ls && Ls < rc[q] + cc[q]) {                    \
                const u64 key = kc[q];                                                        \
                BODY                                                                          \
            }                                                                                 \
        }                                                                                     \
    } else {                                                                                  \
        for (int j = tid; j < H; j += PLAN_THREADS) {                                         \
            if (!(cnt[j] > 0 && rho[j] <= Ls && Ls < rho[j] + cnt[j])) continue;              \
            const u64 key = tie_key(seed, 1u, (unsigned)j, (unsigned)Ls);                     \
            BODY                                                                              \
        }                                                                                     \
    }
        prefix = 0;
        u64 pmask = 0;
        int need = r;
        int left = (int)tsize;  // keys matching the prefix
        if (listed && ntk > 0 && ntk <= PLAN_COUNT_MAX) {
            // few keys: each key's rank is the number of smaller ones (keys
            // of distinct references differ); the one of rank r - 1 is the
            // threshold, found in one pass instead of radix passes. Key e's
            // comparisons are split into `slices` ranges over all threads,
            // the partial counts summed in LDS (the bins are free here).
            const int slices = PLAN_THREADS / ntk;
            const int chunk = (ntk + slices - 1) / slices;
            const int sl = tid / ntk, e = tid - sl * ntk;
            unsigned *rank_of = hist;
            if (tid < ntk) rank_of[tid] = 0;
            lds_barrier();
            if (sl < slices) {
                const u64 mine = t_key[e];
                const int v0 = sl * chunk, v1 = min(ntk, v0 + chunk);
                unsigned part = 0;
#pragma unroll 8
                for (int v = v0; v < v1; ++v) part += t_key[v] < mine;
                if (part) atomicAdd(&rank_of[e], part);
            }
            lds_barrier();
            if (tid < ntk && rank_of[tid] == (unsigned)(r - 1)) cand_thr[0] = t_key[tid];
            lds_barrier();
            prefix = uniform(cand_thr[0]);
            pmask = ~0ull;
            left = 0;
        }
        for (int shift = 52; left > 64; shift = shift >= 12 ? shift - 12 : 0) {
            const int bits = shift >= 4 ? 12 : 4;
            const unsigned dmask = (1u << bits) - 1u;
            for (int q = tid; q < PLAN_BINS; q += PLAN_THREADS) hist[q] = 0;
            lds_barrier();
            PLAN_KEYS({
                if ((key & pmask) == prefix) atomicAdd(&hist[(key >> shift) & dmask], 1u);
            })
            lds_barrier();
            // wave w scans bins 256w .. 256w + 255 (four per lane)
            int h[4], sum = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) { h[q] = (int)hist[wv * 256 + 4 * lane + q]; sum += h[q]; }
            const int incl = wave_incl_scan(sum);
            if (lane == 63) wtot[wv] = incl;
            lds_barrier();
            int before = 0;
            for (int v = 0; v < wv; ++v) before += wtot[v];
            before = uniform(before);
            const int mine = uniform(__builtin_amdgcn_readlane(incl, 63));
            if (before < need && need <= before + mine) {
                const u64 reach = ballot(before + incl >= need);
                const int L = __ffsll((long long)reach) - 1;
                int acc = before + uniform(__builtin_amdgcn_readlane(incl - sum, L));
                int d = wv * 256 + 4 * L + 3, cnt_d = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int hq = uniform(__builtin_amdgcn_readlane(h[q], L));
                    if (acc + hq >= need) { d = wv * 256 + 4 * L + q; cnt_d = hq; break; }
                    acc += hq;
                }
                if (lane == 0) {
                    s_sel[0] = d;
                    s_sel[1] = need - acc;
                    s_sel[2] = cnt_d;
                }
            }
            lds_barrier();
            prefix |= (u64)uniform(s_sel[0]) << shift;
            pmask |= (u64)dmask << shift;
            need = uniform(s_sel[1]);
            left = uniform(s_sel[2]);
            if (shift == 0) break;  // every bit fixed: the key itself
        }
        if (pmask != ~0ull) {
            // at most 64 keys share the prefix: gather them, one wave ranks them
            if (tid == 0) s_sel[3] = 0;
            lds_barrier();
            PLAN_KEYS({
                if ((key & pmask) == prefix) cand[atomicAdd(&s_sel[3], 1)] = key;
            })
            lds_barrier();
            if (wv == 0) {
                const int n = uniform(s_sel[3]);
                const u64 mykey = lane < n ? cand[lane] : ~0ull;
                int rank = 0;
                for (int t = 0; t < n; ++t) {
                    const u64 other = read_lane_u64(mykey, t);
                    rank += other < mykey;
                }
                const u64 hit = ballot(lane < n && rank == need - 1);
                if (lane == 0) cand_thr[0] = read_lane_u64(mykey, __ffsll((long long)hit) - 1);
            }
            lds_barrier();
            prefix = uniform(cand_thr[0]);
        }
#undef PLAN_KEYS
    }
    // per-reference pick counts: up to level L*, plus one at L* for the r
    // least keys of T (members of a listed T are written from the list)
    if (listed) {
        // members of T are written from the list below; no key is hashed here
        PLAN_FOR({
            const bool in_t = cj > 0 && rj <= Ls && Ls < rj + cj;
            if (!in_t) tpick[j] = (int)min((long long)cj, max(0ll, (long long)Ls - rj));
        })
    } else {
        PLAN_FOR({
            const bool in_t = r > 0 && cj > 0 && rj <= Ls && Ls < rj + cj;
            int t = (int)min((long long)cj, max(0ll, (long long)Ls - rj));
            if (in_t && (every || tie_key(seed, 1u, (unsigned)j, (unsigned)Ls) <= prefix)) t += 1;
            tpick[j] = t;
        })
    }
#undef PLAN_FOR
    for (int e = tid; e < ntk; e += PLAN_THREADS)
        tpick[t_ref[e]] = Ls - t_rho[e] + (t_key[e] <= prefix ? 1 : 0);
    if (wv == 0) {
        ctrl->all_pick = 0;
        ctrl->lstar = Ls;
        ctrl->rpick = r;
        ctrl->fl_total = (int)total;
    }
}

// Also counts the members of S per compaction tile (one atomic per wave).
__global__ __launch_bounds__(256) void k_niche_scatter(BatchView bv) {
    const Local L = locate(bv.pt_pref, bv.B);
    CInst &I = bv.tab[L.b];
    const int x = L.i;
    const int l = I.front_info[0];
    const int rk = x < I.M ? I.rank[x] : -1;
    const u64 in_s = ballot(rk >= 0 && rk < l);
    if (lane_id() == 0 && in_s != 0) atomicAdd(&I.P.tcnt[x / COMPACT_TILE], __popcll(in_s));
    if (rk != l) return;
    const int p = I.pi[x];
    if (p < 0 || p >= I.H) return;
    const int slot = atomicAdd(&I.P.fill[p], 1);
    I.P.members[I.P.off[p] + slot] = x;
}

// Makes every lane's earlier LDS and global writes visible to the other lanes
// of the wave before any later read.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Ascending bitonic sort of buf[0..n) by one wave; positions >= n act as +inf
// (the "flip then half-clean" form needs no explicit padding). Block sizes
// are powers of two, so block and position come from shifts and masks; the
// compare-exchanges of one stage are independent, and up to four per lane
// are loaded before any is stored.
__device__ void wave_sort(int *buf, int n) {
    const int lane = lane_id();
    int lp = 0;
    while ((1 << lp) < n) ++lp;
    const int half_n = (1 << lp) >> 1;  // compare-exchanges per stage
    auto stage = [&](auto pair_of) {
        for (int i0 = lane; i0 < half_n; i0 += 256) {
            int a[4], b[4], va[4], vb[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = i0 + 64 * q;
                pair_of(i, a[q], b[q]);
                const bool ok = i < half_n && b[q] < n;
                va[q] = ok ? buf[a[q]] : 0;
                vb[q] = ok ? buf[b[q]] : 0;
                if (!ok) b[q] = -1;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (b[q] >= 0 && va[q] > vb[q]) {
                    buf[a[q]] = vb[q];
                    buf[b[q]] = va[q];
                }
            }
        }
        wave_sync();
    };
    for (int ls = 1; ls <= lp; ++ls) {
        // flip: i against the mirror partner in its block of 2^ls
        const int hs = ls - 1;
        stage([&](int i, int &a, int &b) {
            const int blk = i >> hs, pos = i & ((1 << hs) - 1);
            a = (blk << ls) + pos;
            b = (blk << ls) + (1 << ls) - 1 - pos;
        });
        for (int lh = ls - 2; lh >= 0; --lh) {
            stage([&](int i, int &a, int &b) {
                const int blk = i >> lh, pos = i & ((1 << lh) - 1);
                a = (blk << (lh + 1)) + pos;
                b = a + (1 << lh);
            });
        }
    }
}

// Position of the k-th (0-based) set bit of w.
__device__ __forceinline__ int select_bit(u64 w, int k) {
    int pos = 0;
#pragma unroll
    for (int width = 32; width >= 1; width >>= 1) {
        const u64 lowmask = (width == 64) ? ~0ull : ((1ull << width) - 1);
        const int c = __popcll(w & lowmask);
        if (k >= c) { k -= c; w >>= width; pos += width; }
    }
    return pos;
}

// One wave per reference (4 per workgroup). Segments up to PICK_CAP are
// sorted and tracked in LDS; longer ones in place in global memory.
// Grid: all instances' padded reference ranges, four references per block.
// ORDER (the cache-tensor baseline): every candidate of the reference is
// picked, level after level, and the picks are written in that order to its
// row of the cache tensor (qrow, the reference's segment of the CSR) instead
// of being marked selected.
// Sorts a reference's candidate segment ascending, then makes its picks at
// levels rj .. rj + t - 1. buf and rem are the segment and its remaining-set
// words, either in LDS or in global memory: each call site passes pointers
// of one kind, so that after inlining every access has a known address space
// (no flat accesses).
template <bool ORDER>
__device__ __forceinline__ void pick_sorted(int *buf, u64 *rem, int c, int t, int rj, int j,
                                            u64 seed, const float *__restrict__ dist,
                                            int *picked, int *tcnt, int *qrow) {
    const int lane = lane_id();
    int emitted = 0;  // ORDER: picks written so far
    // records pick x (lane 0)
    auto emit = [&](int x) {
        if (ORDER) {
            qrow[emitted++] = x;
        } else {
            picked[x] = 1;
            atomicAdd(&tcnt[x / COMPACT_TILE], 1);
        }
    };
    wave_sort(buf, c);
    const int nw = (c + 63) / 64;
    if (t >= PICK_DECODE_MIN && t <= PICK_DECODE_MAX) {
        // Every pick's rank among the candidates still remaining when it is
        // made is known in advance: the nearest candidate's position at level
        // 0, else key(seed, 2, j, L) mod (c - p) for pick p at level L. The
        // ranks form a Lehmer code, decoded for all picks at once (one per
        // lane): pick i's position is its rank, raised by one for each
        // earlier pick j (taken from i - 1 down to 0) whose rank is at most
        // the running value (re-inserting pick j at its rank shifts the
        // later ranks by one).
        int pos_near = 0;
        if (rj == 0) {
            u64 best = ~0ull;
#pragma unroll 4
            for (int i = lane; i < c; i += 64) {
                const int x = buf[i];
                const u64 k = ((u64)__float_as_uint(dist[x]) << 32) | (unsigned)i;
                best = k < best ? k : best;
            }
            pos_near = (int)(unsigned)(wave_min_u64(best) & 0xffffffffull);
        }
        constexpr int NB = PICK_DECODE_MAX / 64;
        int kk[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int p = b * 64 + lane;
            kk[b] = 0;
            if (b * 64 < t && p < t)  // (the first test is uniform)
                kk[b] = rj + p == 0 ? pos_near
                                    : (int)(tie_key(seed, 2u, (unsigned)j, (unsigned)(rj + p)) %
                                            (u64)(c - p));
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (b * 64 >= t) break;  // uniform
            int r = kk[b];
#pragma unroll
            for (int q = 63; q >= 0; --q) {
                const int kq = __builtin_amdgcn_readlane(kk[b], q);
                r += (q < lane && kq <= r) ? 1 : 0;
            }
#pragma unroll
            for (int b2 = b - 1; b2 >= 0; --b2) {
#pragma unroll
                for (int q = 63; q >= 0; --q) {
                    const int kq = __builtin_amdgcn_readlane(kk[b2], q);
                    r += kq <= r ? 1 : 0;
                }
            }
            const int n = min(64, t - b * 64);
            if (lane < n && r < c) {
                const int x = buf[r];
                if (ORDER) {
                    qrow[b * 64 + lane] = x;
                } else {
                    picked[x] = 1;
                    atomicAdd(&tcnt[x / COMPACT_TILE], 1);
                }
            }
        }
        return;
    }
    if (nw <= 64) {
        // Up to 4096 candidates: lane w holds word w of the remaining set in a
        // register, and the pick ranks of 64 levels at a time are computed one
        // per lane (they depend on the level only).
        const int v0 = c - lane * 64;
        u64 myrem = lane < nw ? (v0 >= 64 ? ~0ull : ((1ull << v0) - 1)) : 0ull;
        int own = __popcll(myrem);
        // exclusive prefix of the remaining counts by lane, kept current
        // after every removal (no scan per pick)
        int excl = wave_incl_scan(own) - own;
        int kk_lane = 0, kk_base = -1;
        // the positions picked so far, lane p % 64 holding pick p, written out
        // 64 at a time in parallel (off the pick-to-pick chain)
        int mypos = -1, npend = 0;
        auto flush = [&]() {
            if (lane < npend) {
                const int x = buf[mypos];
                if (ORDER) {
                    qrow[emitted + lane] = x;
                } else {
                    picked[x] = 1;
                    atomicAdd(&tcnt[x / COMPACT_TILE], 1);
                }
            }
            emitted += npend;
            npend = 0;
            mypos = -1;
        };
        for (int lev = rj; lev < rj + t; ++lev) {
            int pos;
            if (lev == 0) {
                // first pick of a reference at niche count 0: the nearest candidate
                u64 best = ~0ull;
#pragma unroll 4
                for (int i = lane; i < c; i += 64) {
                    const int x = buf[i];
                    const u64 k = ((u64)__float_as_uint(dist[x]) << 32) | (unsigned)i;
                    best = k < best ? k : best;
                }
                best = wave_min_u64(best);
                pos = (int)(unsigned)(best & 0xffffffffull);
            } else {
                if (kk_base < 0 || lev - kk_base >= 64) {
                    kk_base = lev;
                    const int lv = lev + lane;
                    kk_lane = lv < rj + t ? (int)(tie_key(seed, 2u, (unsigned)j, (unsigned)lv) %
                                                  (u64)(c - (lv - rj)))
                                          : 0;
                }
                const int kk = __builtin_amdgcn_readlane(kk_lane, lev - kk_base);
                const u64 owner = ballot(excl <= kk && kk < excl + own);
                if (owner == 0) break;  // unreachable while the counts are consistent
                const int L = __ffsll((long long)owner) - 1;
                // the word and its prefix on the owning lane, the bit on the
                // scalar unit
                const u64 w = ((u64)(unsigned)__builtin_amdgcn_readlane((int)(myrem >> 32), L) << 32) |
                              (unsigned)__builtin_amdgcn_readlane((int)myrem, L);
                const int base = __builtin_amdgcn_readlane(excl, L);
                pos = L * 64 + select_bit(w, kk - base);
            }
            if (pos < 0 || pos >= c) break;
            // remove position pos: its word's lane loses one, later lanes'
            // prefixes drop by one
            const int lw = pos >> 6;
            if (lane == lw) {
                myrem &= ~(1ull << (pos & 63));
                own -= 1;
            }
            if (lane > lw) excl -= 1;
            if (lane == npend) mypos = pos;
            if (++npend == 64) flush();
        }
        flush();
        return;
    }
    for (int w = lane; w < nw; w += 64) {
        const int v = c - w * 64;
        rem[w] = v >= 64 ? ~0ull : ((1ull << v) - 1);
    }
    // lane L owns words [L*s, (L+1)*s) and keeps their population count
    const int s = (nw + 63) / 64;
    int own = 0;
    for (int w = lane * s; w < min(nw, (lane + 1) * s); ++w) own += __popcll(rem[w]);
    wave_sync();
    for (int lev = rj; lev < rj + t; ++lev) {
        const int remaining = c - (lev - rj);
        int pos;
        if (lev == 0) {
            // first pick of a reference at niche count 0: the nearest candidate
            u64 best = ~0ull;
#pragma unroll 4
            for (int i = lane; i < c; i += 64) {
                const int x = buf[i];
                const u64 k = ((u64)__float_as_uint(dist[x]) << 32) | (unsigned)i;
                best = k < best ? k : best;
            }
            best = wave_min_u64(best);
            pos = (int)(unsigned)(best & 0xffffffffull);
        } else {
            const int kk = (int)(tie_key(seed, 2u, (unsigned)j, (unsigned)lev) % (u64)remaining);
            const int incl = wave_incl_scan(own);
            const int excl = incl - own;
            const u64 owner = ballot(excl <= kk && kk < incl);
            if (owner == 0) break;  // unreachable while the counts are consistent
            const int L = __ffsll((long long)owner) - 1;
            int found = 0;
            if (lane == L) {
                int k2 = kk - excl;
                for (int w = lane * s; w < min(nw, (lane + 1) * s); ++w) {
                    const int pc = __popcll(rem[w]);
                    if (k2 < pc) { found = w * 64 + select_bit(rem[w], k2); break; }
                    k2 -= pc;
                }
            }
            pos = __builtin_amdgcn_readlane(found, L);
        }
        if (pos < 0 || pos >= c) break;
        // remove position pos
        if (lane == 0) rem[pos >> 6] &= ~(1ull << (pos & 63));
        if (lane == (pos >> 6) / s) own -= 1;
        if (lane == 0) emit(buf[pos]);
        wave_sync();
    }
}

template <bool ORDER>
__global__ __launch_bounds__(256) void k_niche_pick(BatchView bv) {
    __shared__ int s_buf[4][PICK_CAP];
    __shared__ u64 s_rem[4][PICK_CAP / 64];
    const int base = uniform((int)(blockIdx.x * 4));
    const int b = uniform(find_range(bv.ref_pref, bv.B, base));
    CInst &I = bv.tab[b];
    const int *__restrict__ rho = I.P.rho;
    const int *__restrict__ cnt = I.P.cnt;
    const int *__restrict__ off = I.P.off;
    const int *__restrict__ tpick = I.P.tpick;
    const float *__restrict__ dist = I.dist;
    const u64 seed = I.seed;
    int *members = I.P.members;
    u64 *remain_g = I.P.remain;
    int *picked = I.P.picked;
    int *tcnt = I.P.tcnt;
    const int wv = threadIdx.x >> 6;
    const int lane = lane_id();
    const int j = base - bv.ref_pref[b] + wv;
    if (j >= I.H) return;
    const int t = ORDER ? cnt[j] : tpick[j];
    if (t <= 0) return;
    const int c = cnt[j];
    int *seg = members + off[j];
    int *qrow = I.P.qrow + off[j];
    int emitted = 0;  // ORDER: picks written so far
    // records pick x (lane 0)
    auto emit = [&](int x) {
        if (ORDER) {
            qrow[emitted++] = x;
        } else {
            picked[x] = 1;
            atomicAdd(&tcnt[x / COMPACT_TILE], 1);
        }
    };
    if (!ORDER && t >= c) {
        for (int i = lane; i < c; i += 64) {
            const int x = seg[i];
            picked[x] = 1;
            atomicAdd(&tcnt[x / COMPACT_TILE], 1);
        }
        return;
    }
    const int rj = rho[j];
    if (t == 1 && rj == 0) {
        // a single pick at niche count 0: the nearest candidate
        u64 best = ~0ull;
        for (int i = lane; i < c; i += 64) {
            const int x = seg[i];
            const u64 k = ((u64)__float_as_uint(dist[x]) << 32) | (unsigned)x;
            best = k < best ? k : best;
        }
        best = wave_min_u64(best);
        if (lane == 0) emit((int)(unsigned)(best & 0xffffffffull));
        return;
    }
    if (c <= PICK_CAP) {
#pragma unroll 8
        for (int i = lane; i < c; i += 64) s_buf[wv][i] = seg[i];
        wave_sync();
        pick_sorted<ORDER>(s_buf[wv], s_rem[wv], c, t, rj, j, seed, dist, picked, tcnt, qrow);
    } else {
        pick_sorted<ORDER>(seg, remain_g + (off[j] >> 6) + j, c, t, rj, j, seed, dist, picked,
                           tcnt, qrow);
    }
}

// ------------------------------------------------- cache-tensor baseline
//
// The paper's own niche fill (Algorithm 2, nearest selection and the random
// selection loop over the cache tensor Q), for an A/B comparison with the
// closed form above; same inputs, same keys, the same selection. Q's row j
// holds the candidates of reference j in the order reference j picks them
// (the nearest first at niche count 0, then keyed picks; k_niche_pick<true>),
// so the row position s_j is the next pick. The rows are the reference's CSR
// segment (the paper pads them to a dense w x n tensor, which only changes
// the memory used). Then one workgroup per instance runs the loop: find the
// least niche count among references with candidates left, let every
// reference at that count take its next row entry, update the counts, until
// K are taken; the last iteration keeps the references with the least tag-1
// keys (the paper truncates the last selection in its shuffled reference
// order).

// Exclusive scan of c over the references (the CSR offsets of Q's rows), one
// workgroup per instance.
__global__ __launch_bounds__(PLAN_THREADS) void k_ct_offsets(BatchView bv) {
    CInst &I = bv.tab[blockIdx.x];
    __shared__ int wsum[PLAN_WAVES];
    __shared__ int s_carry;
    const int tid = threadIdx.x, wv = tid >> 6, lane = lane_id();
    const int H = I.H;
    if (tid == 0) s_carry = 0;
    lds_barrier();
    for (int j0 = 0; j0 < H; j0 += PLAN_THREADS) {
        const int j = j0 + tid;
        const int c = j < H ? I.P.cnt[j] : 0;
        const int incl = wave_incl_scan(c);
        if (lane == 63) wsum[wv] = incl;
        lds_barrier();
        int before = uniform(s_carry);
        for (int v = 0; v < wv; ++v) before += wsum[v];
        if (j < H) I.P.off[j] = before + incl - c;
        lds_barrier();
        if (tid == PLAN_THREADS - 1) s_carry = before + incl;
        lds_barrier();
    }
    if (tid == 0) I.P.off[H] = s_carry;
}

__device__ __forceinline__ long long block_min_ll(long long v, long long *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, (long long)__shfl_xor(v, o, 64));
    lds_barrier();
    if (lane_id() == 0) red[threadIdx.x >> 6] = v;
    lds_barrier();
    long long m = LLONG_MAX;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) m = min(m, red[i]);
    return uniform(m);
}

// The selection loop. Reference j's state: its niche count lev_j = rho_j +
// s_j and its candidates left, left_j = c_j - s_j (s_j picks made); it takes
// part while left_j > 0. The state lives in LDS when H <= CT_LDS_REFS, else
// in workspace arrays (tpick, fill: free after the scatter).
constexpr int CT_LDS_REFS = 12288;

template <bool IN_LDS>
__device__ void ct_loop(CInst &I, int *lev, int *left) {
    __shared__ long long red[PLAN_WAVES];
    __shared__ unsigned hist[256];
    __shared__ int s_sel[2];
    const int tid = threadIdx.x;
    const int H = I.H;
    const u64 seed = I.seed;
    const int *__restrict__ cnt = I.P.cnt;
    const int *__restrict__ off = I.P.off;
    const int *__restrict__ qrow = I.P.qrow;
    int *picked = I.P.picked;
    int *tcnt = I.P.tcnt;
    const long long K = uniform(I.front_info[2]);
    for (int j = tid; j < H; j += PLAN_THREADS) {
        lev[j] = I.P.rho[j];
        left[j] = cnt[j];
    }
    lds_barrier();  // each thread reads back only its own references
    long long taken = 0;
    while (taken < K) {
        // mark tensor u: the references of least niche count with candidates left
        long long lmin = LLONG_MAX;
        long long nu = 0;
        for (int j = tid; j < H; j += PLAN_THREADS)
            if (left[j] > 0) lmin = min(lmin, (long long)lev[j]);
        lmin = block_min_ll(lmin, red);
        if (lmin == LLONG_MAX) {
            // fewer candidates than K: an inconsistent input
            if (tid == 0) atomicOr(&I.P.ctrl->status, ST_INTERNAL);
            break;
        }
        for (int j = tid; j < H; j += PLAN_THREADS) nu += (left[j] > 0 && lev[j] == lmin);
        nu = block_sum_ll(nu, red);
        // the last iteration keeps the r least tag-1 keys of u: threshold by
        // radix select, 8 bits per pass from the top
        const bool trunc = taken + nu > K;
        u64 thr = ~0ull;
        if (trunc) {
            int need = (int)(K - taken);
            u64 prefix = 0, pmask = 0;
            for (int shift = 56; shift >= 0; shift -= 8) {
                for (int q = tid; q < 256; q += PLAN_THREADS) hist[q] = 0;
                lds_barrier();
                for (int j = tid; j < H; j += PLAN_THREADS) {
                    if (!(left[j] > 0 && lev[j] == lmin)) continue;
                    const u64 key = tie_key(seed, 1u, (unsigned)j, (unsigned)lmin);
                    if ((key & pmask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
                }
                lds_barrier();
                if (tid < 64) {
                    int d, rest;
                    hist_digit(hist, need, d, rest);
                    if (tid == 0) {
                        s_sel[0] = d;
                        s_sel[1] = rest;
                    }
                }
                lds_barrier();
                prefix |= (u64)uniform(s_sel[0]) << shift;
                pmask |= 0xffull << shift;
                need = uniform(s_sel[1]);
                lds_barrier();  // s_sel and hist are reused
            }
            thr = prefix;  // the r-th least key itself (keys of distinct references differ)
        }
        // select Q[j][s_j] for the marked references; their niche counts and
        // row positions advance
        for (int j = tid; j < H; j += PLAN_THREADS) {
            const int lj = left[j];
            if (!(lj > 0 && lev[j] == lmin)) continue;
            if (trunc && tie_key(seed, 1u, (unsigned)j, (unsigned)lmin) > thr) continue;
            const int x = qrow[off[j] + cnt[j] - lj];
            picked[x] = 1;
            atomicAdd(&tcnt[x / COMPACT_TILE], 1);
            left[j] = lj - 1;
            lev[j] = (int)lmin + 1;
        }
        lds_barrier();
        taken = trunc ? K : taken + nu;
    }
}

__global__ __launch_bounds__(PLAN_THREADS) void k_ct_loop(BatchView bv) {
    __shared__ int s_lev[CT_LDS_REFS], s_left[CT_LDS_REFS];
    CInst &I = bv.tab[blockIdx.x];
    if (uniform(I.H) <= CT_LDS_REFS) ct_loop<true>(I, s_lev, s_left);
    else ct_loop<false>(I, I.P.tpick, I.P.fill);
}

// Compaction of {x : rank[x] < l or picked[x]} in ascending order, one
// workgroup per tile of COMPACT_TILE points. The scatter and pick kernels
// counted the selected points of every tile, so a tile's first output
// position is the sum of the counts before it (one wave adds them up); a
// ballot per wave and the wave counts give every point's position.
// Grid: all instances' padded point ranges.
static_assert(COMPACT_TILE == PT_ALIGN, "a workgroup of the point grid is one tile");
__global__ __launch_bounds__(COMPACT_TILE) void k_compact(BatchView bv) {
    __shared__ int s_base;
    __shared__ int wcnt[COMPACT_TILE / 64];
    const Local L = locate(bv.pt_pref, bv.B);
    CInst &I = bv.tab[L.b];
    const int x = L.i;
    const int M = I.M, N = I.N, l = I.front_info[0];
    const int t = uniform(x / COMPACT_TILE);
    if (t * COMPACT_TILE >= M) return;  // a tile of padding only
    const int wv = threadIdx.x >> 6;
    const int lane = lane_id();
    const int *tcnt = I.P.tcnt;
    if (wv == 0) {
        int sum = 0;
        for (int u = lane; u < t; u += 64) sum += tcnt[u];
        sum = wave_sum(sum);
        if (lane == 0) s_base = sum;
    }
    const int rk = x < M ? I.rank[x] : -1;
    const bool sel = x < M && ((rk >= 0 && rk < l) || I.P.picked[x] != 0);
    const u64 fl = ballot(sel);
    if (lane == 0) wcnt[wv] = __popcll(fl);
    lds_barrier();
    int pos = s_base;
    for (int v = 0; v < wv; ++v) pos += wcnt[v];
    pos += mbcnt(fl);
    if (sel && pos < N) I.selected[pos] = x;
    // the last tile checks the total against N
    if (threadIdx.x == 0 && (t + 1) * COMPACT_TILE >= M) {
        int total = s_base;
        for (int v = 0; v < COMPACT_TILE / 64; ++v) total += wcnt[v];
        if (total != N) atomicOr(&I.P.ctrl->status, ST_INTERNAL);
    }
}

hipError_t launch_niche(const HostPlan &hp, const BatchView &bv, hipStream_t s) {
    const unsigned pblocks = (unsigned)(hp.npt / 256);
    const unsigned rblocks = (unsigned)(hp.nref / 4);
    if (!(bv.run & RUN_ASSOC))
        NSGA3_LAUNCH("niche_count", k_niche_count, dim3(pblocks), dim3(256), 0, s, bv);
    if (bv.run & RUN_CACHE_TENSOR) {
        NSGA3_LAUNCH("ct_offsets", k_ct_offsets, dim3(hp.B), dim3(PLAN_THREADS), 0, s, bv);
        NSGA3_LAUNCH("niche_scatter", k_niche_scatter, dim3(pblocks), dim3(256), 0, s, bv);
        NSGA3_LAUNCH("ct_order", k_niche_pick<true>, dim3(rblocks), dim3(256), 0, s, bv);
        NSGA3_LAUNCH("ct_loop", k_ct_loop, dim3(hp.B), dim3(PLAN_THREADS), 0, s, bv);
    } else {
        NSGA3_LAUNCH("niche_plan", k_niche_plan, dim3(hp.B), dim3(PLAN_THREADS), 0, s, bv);
        NSGA3_LAUNCH("niche_scatter", k_niche_scatter, dim3(pblocks), dim3(256), 0, s, bv);
        NSGA3_LAUNCH("niche_pick", k_niche_pick<false>, dim3(rblocks), dim3(256), 0, s, bv);
    }
    NSGA3_LAUNCH("compact", k_compact, dim3(hp.npt / 256), dim3(COMPACT_TILE), 0, s, bv);
    return hipGetLastError();
}

}  // namespace nsga3
