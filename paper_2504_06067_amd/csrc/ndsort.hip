// Non-dominated sorting (paper Sec. II-C; Algorithm 1 "Non-dominated-sort")
// as a bit-packed dominance matrix followed by front peeling, for a batch of
// independent instances.
//
// Dominance matrix layout ("word-major"): mask[w * Mp + j] is a 64-bit word
// whose bit b is set iff point 64*w + b dominates point j. A wave of 64
// consecutive j therefore reads or writes 512 contiguous bytes.
//
// Kernels:
//   k_init       per instance: control block, peel counters, front_info
//   k_prep       points: tile-major objective copy (+inf padding), finiteness,
//                dominator counts, ranks, alive set of front 0, niche flags;
//                references: unit directions and their check, niche counters
//   k_dominance  triangle of 64x64 tiles; both directions from one set of 2m
//                compares per pair; fused dominator counts
//   k_peel       fronts of every instance, persistent over all their chunks
#include <utility>

#include "nsga3_internal.h"

namespace nsga3 {

long long dominance_items(int W, int G_) {
    const long long G = G_, q = W / G, s = W % G;
    return (long long)W + G * q * (q - 1) / 2 + q * s;
}

__global__ __launch_bounds__(256) void k_init(BatchView bv) {
    CInst &I = bv.tab[blockIdx.x];
    Ctrl *ctrl = I.P.ctrl;
    const int t = threadIdx.x;
    if (t == 0) {
        ctrl->status = 0;
        ctrl->list_count = 0;
        if (bv.run & RUN_ND) {
            // a defined value even if the peel stops on an internal error
            I.front_info[0] = 0;
            I.front_info[1] = 0;
            I.front_info[2] = I.n_stop;
            I.front_info[3] = 0;
        }
    }
    if (blockIdx.x == 0 && t == 0) *bv.ticket = 0;
    if (t < NSGA3_MAX_OBJECTIVES) {
        ctrl->zmin_enc[t] = 0xffffffffu;
        ctrl->fmax_enc[t] = 0u;
        ctrl->ext_key[t] = ~0ull;
    }
    if (bv.run & RUN_ND)
        for (int i = t; i < 3 * PEEL_SLOT; i += blockDim.x) I.P.facc[i] = 0;
}

// Grid: [all instances' padded points][all instances' padded references].
__global__ __launch_bounds__(256) void k_prep(BatchView bv, int npt) {
    const bool points = (int)(blockIdx.x * blockDim.x) < npt;
    if (points) {
        const Local L = locate(bv.pt_pref, bv.B);
        CInst &I = bv.tab[L.b];
        const int j = L.i, M = I.M, m = I.m, Mp = I.Mp;
        bool bad = false;
        if (j < Mp && (bv.run & RUN_ND)) {
            for (int k = 0; k < m; ++k) {
                float v = INFINITY;
                if (j < M) {
                    v = I.F[(size_t)j * m + k];
                    bad |= !isfinite(v);
                }
                I.P.ft[((size_t)(j >> 6) * m + k) * 64 + (j & 63)] = v;
            }
            I.P.nd[j] = 0;
            if (j < M) I.rank[j] = NSGA3_UNRANKED;
            if ((j & 63) == 0) {
                const int valid = M - j;
                I.P.alive[(size_t)(j >> 6) * ALIVE_PAD] =
                    valid >= 64 ? ~0ull : (valid <= 0 ? 0ull : ((1ull << valid) - 1));
            }
        }
        if (j < M && (bv.run & RUN_NICHE)) I.P.picked[j] = 0;
        if (ballot(bad) != 0 && lane_id() == 0) atomicOr(&I.P.ctrl->status, ST_NONFINITE);
    } else {
        const int base = uniform((int)(blockIdx.x * blockDim.x)) - npt;
        const int b = uniform(find_range(bv.ref_pref, bv.B, base));
        CInst &I = bv.tab[b];
        const int t = base - bv.ref_pref[b] + (int)threadIdx.x;
        const int H = I.H, Hp = I.Hp, m = I.m;
        bool bad = false;
        if (t < Hp && (bv.run & RUN_ASSOC)) {
            // unit reference directions; padding repeats the last real one
            const int j = t < H ? t : H - 1;
            float s = 0.0f;
            for (int k = 0; k < m; ++k) {
                const float v = I.Z[(size_t)j * m + k];
                bad |= !(v >= 0.0f) || !isfinite(v);
                s = fmaf(v, v, s);
            }
            bad |= !(s > 0.0f);
            const float inv = bad ? 0.0f : 1.0f / sqrtf(s);
            for (int k = 0; k < m; ++k) I.P.wn[(size_t)k * Hp + t] = I.Z[(size_t)j * m + k] * inv;
        }
        if (t < H && (bv.run & RUN_NICHE)) {
            I.P.rho[t] = 0;
            I.P.cnt[t] = 0;
            I.P.fill[t] = 0;
        }
        if (ballot(bad) != 0 && lane_id() == 0) atomicOr(&I.P.ctrl->status, ST_BADREF);
    }
}

// (a << 1) | bit(lane) for every lane, with the bits taken from a wave mask:
// one v_addc with the mask as carry-in (a + a + carry).
__device__ __forceinline__ unsigned shift_in(unsigned a, u64 mask) {
    unsigned r;
    u64 carry_out;
    asm("v_addc_co_u32 %0, %1, %2, %2, %3" : "=v"(r), "=s"(carry_out) : "v"(a), "s"(mask));
    return r;
}

// The value of lane L (wave-uniform) of a 64-bit register pair.
__device__ __forceinline__ u64 read_lane64(u64 x, int L) {
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)x, L);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)(x >> 32), L);
    return ((u64)hi << 32) | lo;
}

// Lane R of `old` takes the wave-uniform value v.
template <int R>
__device__ __forceinline__ unsigned write_lane(unsigned old, unsigned v) {
    asm("v_writelane_b32 %0, %1, %2" : "+v"(old) : "s"(v), "i"(R));
    return old;
}

// Work items of block rows 0 .. jb - 1 for G = 2^gsh column tiles per item.
__device__ __forceinline__ long long items_before(int jb, int gsh) {
    const long long q = jb >> gsh, s = jb & ((1 << gsh) - 1);
    return (long long)jb + (((q * (q - 1)) >> 1) << gsh) + q * s;
}

// GW consecutive column values of one objective (one scalar load). The
// group width keeps GW * m values within the scalar register budget.
template <int MO>
constexpr int col_group() { return MO <= 4 ? 8 : (MO <= 8 ? 4 : 2); }

template <int GW>
struct alignas(4 * GW) ColV {
    float a[GW];
};

// One compare step against column point i = 64 * ib + R (uniform, objective
// values v[k].a[R % GW]): the wave masks lt = {j : f_i < f_j in some
// objective}, gt = {j : f_i > f_j in some objective} come from 2m compares;
// then
//   i dominates j  <=>  j in lt \ gt   (bit R of lane j's word A)
//   j dominates i  <=>  j in gt \ lt   (the whole mask is row i's word B)
template <int MO, int GW, int R>
__device__ __forceinline__ void dom_step(const ColV<GW> (&v)[MO], const float (&fj)[MO],
                                         unsigned &a_lo, unsigned &a_hi, unsigned &b_lo,
                                         unsigned &b_hi) {
    u64 lt = 0, gt = 0;
#pragma unroll
    for (int k = 0; k < MO; ++k) {
        const float x = v[k].a[R % GW];
        lt |= ballot(x < fj[k]);
        gt |= ballot(x > fj[k]);
    }
    const u64 i_dom_j = lt & ~gt;
    const u64 j_dom_i = gt & ~lt;
    if (R >= 32) a_hi = shift_in(a_hi, i_dom_j);
    else a_lo = shift_in(a_lo, i_dom_j);
    b_lo = write_lane<R>(b_lo, (unsigned)j_dom_i);
    b_hi = write_lane<R>(b_hi, (unsigned)(j_dom_i >> 32));
}

// Column points GW*g + GW - 1 down to GW*g: their values arrive with one
// scalar load per objective.
template <int MO, int GW, int g, int... Is>
__device__ __forceinline__ void dom_group(std::integer_sequence<int, Is...>,
                                          const NSGA3_RO float *fi, const float (&fj)[MO],
                                          unsigned &a_lo, unsigned &a_hi, unsigned &b_lo,
                                          unsigned &b_hi) {
    ColV<GW> v[MO];
#pragma unroll
    for (int k = 0; k < MO; ++k) {
        const NSGA3_RO ColV<GW> &src = *(const NSGA3_RO ColV<GW> *)(fi + k * 64 + GW * g);
#pragma unroll
        for (int q = 0; q < GW; ++q) v[k].a[q] = src.a[q];
    }
    (dom_step<MO, GW, GW * g + GW - 1 - Is>(v, fj, a_lo, a_hi, b_lo, b_hi), ...);
}

// R runs 63 down to 0 so that the shifted-in bit of point 64*ib + R lands at
// bit R (of the high word for R >= 32).
template <int MO, int GW, int... Gs>
__device__ __forceinline__ void dom_tile(std::integer_sequence<int, Gs...>,
                                         const NSGA3_RO float *fi, const float (&fj)[MO],
                                         unsigned &a_lo, unsigned &a_hi, unsigned &b_lo,
                                         unsigned &b_hi) {
    constexpr int NG = 64 / GW;
    (dom_group<MO, GW, NG - 1 - Gs>(std::make_integer_sequence<int, GW>{}, fi, fj, a_lo, a_hi,
                                    b_lo, b_hi),
     ...);
}

// One wave per work item of the instances with m = MO (the group order[gs ..
// gs + gn)): the 64 points of block row jb sit in the lanes (as the dominated
// side j); the item sweeps up to G column blocks ib <= jb, reading the
// column points through the scalar cache.
template <int MO>
__global__ __launch_bounds__(256) void k_dominance(BatchView bv, int gs, int gn,
                                                    long long item0, long long n_items) {
    const int lane = lane_id();
    const long long gitem = uniform(item0 + (long long)blockIdx.x * 4 + (threadIdx.x >> 6));
    if (gitem >= item0 + n_items) return;
    const int gi = uniform(find_range(bv.dom_pref + gs, gn, gitem));
    CInst &I = bv.tab[bv.order[gs + gi]];
    const long long item = gitem - bv.dom_pref[gs + gi];
    const int W = I.W, Mp = I.Mp, G = I.G, gsh = __builtin_ctz((unsigned)G);
    // the objective copy is written by k_prep and only read here: invariant
    // loads, so the column points come through the scalar cache
    const NSGA3_RO float *ft = (const NSGA3_RO float *)I.P.ft;
    u64 *__restrict__ mask = I.P.mask;
    int *__restrict__ nd = I.P.nd;
    // block row: largest jb with items_before(jb) <= item
    int lo = 0, hi = W;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (items_before(mid, gsh) <= item) lo = mid;
        else hi = mid;
    }
    const int jb = lo;
    const int g = (int)(item - items_before(jb, gsh));
    const int ib0 = g * G;
    const int ib1 = min(ib0 + G, jb + 1);

    const size_t jglob = (size_t)jb * 64 + lane;
    float fj[MO];
#pragma unroll
    for (int k = 0; k < MO; ++k) fj[k] = ft[((size_t)jb * MO + k) * 64 + lane];

    int cnt_j = 0;
    for (int ib = ib0; ib < ib1; ++ib) {
        unsigned a_lo = 0, a_hi = 0, b_lo = 0, b_hi = 0;
        const NSGA3_RO float *fi = ft + (size_t)ib * MO * 64;
        constexpr int GW = col_group<MO>();
        dom_tile<MO, GW>(std::make_integer_sequence<int, 64 / GW>{}, fi, fj, a_lo, a_hi, b_lo, b_hi);
        const u64 A = ((u64)a_hi << 32) | a_lo;
        mask[(size_t)ib * Mp + jglob] = A;
        cnt_j += __popcll(A);
        if (ib != jb) {
            const u64 B = ((u64)b_hi << 32) | b_lo;
            mask[(size_t)jb * Mp + (size_t)ib * 64 + lane] = B;
            const int c = __popcll(B);
            if (c) atomicAdd(&nd[ib * 64 + lane], c);
        }
    }
    if (cnt_j) atomicAdd(&nd[jglob], cnt_j);
}

// Front peeling.
//
// Chunk c of an instance holds its 64 points 64c .. 64c+63. Front 0 is
// {j : no dominator} (fused counts of the dominance kernel). A point j alive
// at front k > 0 belongs to it iff no alive point dominates it. Fronts after
// the first are found with witnesses: every alive point keeps one alive
// dominator (its witness) and is re-examined only once its witness has been
// ranked. The re-examination resumes the scan of j's row at the witness's
// word: the words before it held no alive dominator when they were scanned,
// and the alive set only shrinks. Over the whole peel each row is read about
// once. The scans read a row-major copy of the dominance matrix (row j = the W
// words of point j's dominators), which each workgroup writes for its own
// chunks when their instance starts front 1; an instance whose front 0
// already fills N never builds it. The peel of an instance stops once its
// ranked fronts hold n_stop points.
//
// Scheduling. While ranking front 0, workgroups claim chunks (of any
// instance) from a ticket counter until every chunk is claimed; a workgroup
// then owns its chunks for all later fronts and processes them front by
// front. Only running workgroups claim, and no workgroup waits before all
// chunks are claimed and ranked for front 0; later waits are for lower fronts
// of chunks owned by running workgroups, so every wait ends. A workgroup
// records at most PEEL_OWN_CAP chunks; if every running workgroup were full
// the front-0 wait would time out into an error status.
//
// Completion. Per front, chunk c adds (points ranked << 32) + 1 to shard
// counter c % PEEL_SHARDS of its instance (a fire-and-forget atomic); a
// waiting workgroup reads the 32 shards with one wave and sums them. Counters
// live in a ring of three front slots per instance; the slot of front k + 1
// is cleared while front k is processed (after front k - 1 completed, nobody
// reads it).
//
// Memory ordering. Alive words and counters are written with agent-scope
// atomic stores, which go to the coherent level; each chunk waits for its
// stores before its counter add. Waiters poll the counters with relaxed
// atomic loads. Alive words are then read with ordinary cached loads: the
// word of each chunk sits alone on a 128-byte line of a per-front slot, so
// no line is written by two workgroups and none is cached before it is read;
// slots are reused only after `ns` fronts, and then an agent-scope acquire
// drops stale copies. The row-major copy and the witnesses of a chunk are
// touched only by its owner.
//
// Control flow is wave-uniform around every workgroup barrier: wave 0 makes
// the scheduling decisions with all its lanes and shares them through LDS.
constexpr int PEEL_WAVES = 8;
constexpr int PEEL_OWN_CAP = 1024;
constexpr int PEEL_LDS_ALIVE = 2048;  // alive words staged in LDS (M <= 131072)

__device__ __forceinline__ u64 *peel_slot(u64 *ring, int k) { return ring + (size_t)(k % 3) * PEEL_SLOT; }

// Alive bitset of front k: slot k % ns of the alive ring.
__device__ __forceinline__ u64 *alive_slot(u64 *aring, int W, int ns, int k) {
    return aring + (size_t)(k % ns) * W * ALIVE_PAD;
}

struct PeelShared {
    int own_b[PEEL_OWN_CAP];    // instance of each owned chunk
    int own_c[PEEL_OWN_CAP];    // chunk within its instance
    int own_cum[PEEL_OWN_CAP];  // points in the instance's fronts seen so far (-1: done)
    union {                     // the transpose (front 1 start) and the scans never overlap
        u64 alive[PEEL_LDS_ALIVE];
        u64 tile[64][65];
    };
    u64 val;
    u64 need;
    u64 newly;
    int flag;
};

// Row-major copy of chunk c's rows: rowm[j][w] = mask[w][j], through a
// padded 64 x 64-word LDS tile (coalesced reads and writes).
__device__ void peel_transpose(CInst &I, int c, PeelShared &sh) {
    const int lane = lane_id();
    const int wv = uniform((int)(threadIdx.x >> 6));
    const int W = I.W, Mp = I.Mp;
    const u64 *__restrict__ mask = I.P.mask;
    u64 *__restrict__ rowm = I.P.rowm;
    for (int w0 = 0; w0 < W; w0 += 64) {
#pragma unroll
        for (int q = 0; q < 64 / PEEL_WAVES; ++q) {
            const int wl = wv * (64 / PEEL_WAVES) + q;
            const int w = w0 + wl;
            sh.tile[wl][lane] = (w < W) ? mask[(size_t)w * Mp + (size_t)c * 64 + lane] : 0ull;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 64 / PEEL_WAVES; ++q) {
            const int r = wv * (64 / PEEL_WAVES) + q;
            const int w = w0 + lane;
            if (w < W) rowm[((size_t)c * 64 + r) * W + w] = sh.tile[lane][r];
        }
        __syncthreads();
    }
    if (wv == 0) I.P.wit[c * 64 + lane] = -1;
}

// Ranks the points of chunk c that are alive at front k and have no alive
// dominator; publishes the chunk's result. All waves take part.
// STAGED: the alive words of front k are copied to LDS (W <= PEEL_LDS_ALIVE);
// a compile-time choice, so that no pointer ever selects between LDS and
// global memory.
template <bool STAGED>
__device__ void peel_chunk_impl(CInst &I, int k, int c, PeelShared &sh) {
    const int lane = lane_id();
    const int wv = uniform((int)(threadIdx.x >> 6));
    const int W = I.W, ns = I.ns;
    const u64 *alive_k = alive_slot(I.P.alive, W, ns, k);
    u64 *alive_n = alive_slot(I.P.alive, W, ns, k + 1);
    const u64 aw = uniform(alive_k[(size_t)c * ALIVE_PAD]);
    const int j = c * 64 + lane;
    u64 newly;
    if (k == 0) {
        newly = aw & ballot(I.P.nd[j] == 0);
    } else {
        constexpr bool staged = STAGED;
        const u64 *__restrict__ rowm = I.P.rowm;
        int *wit = I.P.wit;
        __syncthreads();  // the previous chunk is done with the shared words
        if (staged && aw != 0)
            for (int w = threadIdx.x; w < W; w += blockDim.x) sh.alive[w] = alive_k[(size_t)w * ALIVE_PAD];
        if (wv == 0) sh.newly = 0;
        __syncthreads();
        // points whose witness is still alive stay dominated
        if (wv == 0) {
            bool need = false;
            if ((aw >> lane) & 1ull) {
                const int wj = wit[j];
                if (wj < 0) {
                    need = true;
                } else {
                    const u64 word = staged ? sh.alive[wj >> 6] : alive_k[(size_t)(wj >> 6) * ALIVE_PAD];
                    need = ((word >> (wj & 63)) & 1ull) == 0;
                }
            }
            sh.need = ballot(need);
        }
        __syncthreads();
        const u64 need = uniform(sh.need);
        // wave wv re-examines the needing points wv, wv + PEEL_WAVES, ... (lane
        // order)
        constexpr int PER = 64 / PEEL_WAVES;
        int pl[PER];
        int mine = 0;
        {
            u64 rest = need;
            for (int skip = 0; skip < wv && rest; ++skip) rest &= rest - 1;
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                pl[q] = rest ? __ffsll((long long)rest) - 1 : -1;
                if (rest) {
                    ++mine;
                    for (int skip = 0; skip < PEEL_WAVES && rest; ++skip) rest &= rest - 1;
                }
            }
        }
        // All needing points of the wave search together: each round loads the
        // next 128 words (two per lane) of every point still searching, so the
        // rounds of different points overlap instead of adding up.
        int pos[PER], state[PER], fwi[PER];  // state: 0 searching, 1 found, 2 none, 3 unused
        u64 fw[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            pos[q] = 0;
            fwi[q] = 0;
            fw[q] = 0;
            state[q] = q < mine ? 0 : 3;
            if (q < mine) {
                const int wp = uniform(wit[c * 64 + pl[q]]);
                pos[q] = wp < 0 ? 0 : (wp >> 6);
            }
        }
        for (;;) {
            u64 x0[PER], x1[PER];
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                x0[q] = 0;
                x1[q] = 0;
                if (state[q] == 0) {
                    const u64 *__restrict__ row = rowm + (size_t)(c * 64 + pl[q]) * W;
                    const int w = pos[q] + 2 * lane;
                    if (w < W)
                        x0[q] = row[w] & (staged ? sh.alive[w] : alive_k[(size_t)w * ALIVE_PAD]);
                    if (w + 1 < W)
                        x1[q] = row[w + 1] &
                                (staged ? sh.alive[w + 1] : alive_k[(size_t)(w + 1) * ALIVE_PAD]);
                }
            }
            int searching = 0;
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                if (state[q] != 0) continue;
                const u64 b = ballot((x0[q] | x1[q]) != 0);
                if (b) {
                    const int L = __ffsll((long long)b) - 1;
                    const u64 a0 = read_lane64(x0[q], L);
                    const u64 a1 = read_lane64(x1[q], L);
                    fw[q] = a0 ? a0 : a1;
                    fwi[q] = pos[q] + 2 * L + (a0 ? 0 : 1);
                    state[q] = 1;
                } else {
                    pos[q] += 128;
                    if (pos[q] >= W) state[q] = 2;
                    else searching = 1;
                }
            }
            if (!searching) break;
        }
        // new witness: among the alive dominators in the first word that has
        // any, the one with the most dominators of its own (a proxy for the
        // deepest, which stays alive longest); the loads of all points overlap
        u64 key[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            key[q] = 0;
            const int cand = fwi[q] * 64 + lane;
            if (state[q] == 1 && ((fw[q] >> lane) & 1ull))
                key[q] = ((u64)(unsigned)I.P.nd[cand] << 32) | (unsigned)(~cand);
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            if (state[q] != 1 && state[q] != 2) continue;
            int found = -1;
            if (state[q] == 1) found = (int)~(unsigned)(wave_max_u64(key[q]) & 0xffffffffull);
            const int jp = c * 64 + pl[q];
            if (lane == 0) wit[jp] = found;
            if (found < 0 && lane == 0) atomicOr(&sh.newly, 1ull << pl[q]);
        }
        __syncthreads();
        newly = aw & uniform(sh.newly);
    }
    if (wv == 0) {
        store_relaxed(&alive_n[(size_t)c * ALIVE_PAD], aw & ~newly);
        __builtin_amdgcn_s_waitcnt(0);
        u64 *slot = peel_slot(I.P.facc, k);
        const u64 add = ((u64)__popcll(newly) << 32) | 1ull;
        __hip_atomic_fetch_add(&slot[(c % PEEL_SHARDS) * PEEL_STRIDE], lane == 0 ? add : 0ull,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((newly >> lane) & 1ull) I.rank[j] = k;  // read only by later kernels
    }
}

__device__ __forceinline__ void peel_chunk(CInst &I, int k, int c, PeelShared &sh) {
    if (uniform(I.W) <= PEEL_LDS_ALIVE) peel_chunk_impl<true>(I, k, c, sh);
    else peel_chunk_impl<false>(I, k, c, sh);
}

__global__ __launch_bounds__(64 * PEEL_WAVES) void k_peel(BatchView bv, int nchunk) {
    __shared__ PeelShared sh;
    const int lane = lane_id();
    const int wv = uniform((int)(threadIdx.x >> 6));
    const u64 one = lane == 0 ? 1ull : 0ull;
    // drop cached lines of alive slots read by an earlier call on these workspaces
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");

    // front 0: claim and rank chunks until all are claimed
    int nown = 0;
    for (;;) {
        if (wv == 0) sh.val = uniform(atomicAdd(bv.ticket, one));
        __syncthreads();
        const u64 t = uniform(sh.val);
        __syncthreads();
        if (t >= (u64)nchunk) break;
        const int b = uniform(find_range(bv.chunk_pref, bv.B, (int)t));
        const int c = (int)t - bv.chunk_pref[b];
        peel_chunk(bv.tab[b], 0, c, sh);
        if (wv == 0) {
            sh.own_b[nown] = b;
            sh.own_c[nown] = c;
            sh.own_cum[nown] = 0;
        }
        ++nown;
        if (nown == PEEL_OWN_CAP) break;
    }
    __syncthreads();
    // a workgroup without chunks has nothing left to do; the owners of the
    // chunks report the front fill
    if (nown == 0) return;

    for (int k = 1;; ++k) {
        int active = 0;
        for (int q = 0; q < nown; ++q) {
            const int b = uniform(sh.own_b[q]);
            const int c = uniform(sh.own_c[q]);
            const int cum_prev = uniform(sh.own_cum[q]);
            if (cum_prev < 0) continue;  // this instance finished
            CInst &I = bv.tab[b];
            // wait for front k - 1 of the instance
            if (wv == 0) {
                const u64 *slot = peel_slot(I.P.facc, k - 1);
                u64 v = 0;
                int ok = 1;
                for (unsigned polls = 0;; ++polls) {
                    // lanes 0..31 read one shard each; the wave sums (count, size)
                    const u64 part = lane < PEEL_SHARDS ? load_relaxed(&slot[lane * PEEL_STRIDE]) : 0ull;
                    v = uniform(wave_sum(part));
                    if ((unsigned)(v & 0xffffffffull) >= (unsigned)I.W) break;
                    if (polls == (1u << 26)) { ok = 0; break; }
                    __builtin_amdgcn_s_sleep(2);
                }
                sh.val = v;
                sh.flag = ok;
            }
            __syncthreads();
            const u64 v = uniform(sh.val);
            const int ok = uniform(sh.flag);
            // alive slots are reused only after ns fronts: then cached copies of the
            // slot read ns fronts ago must be dropped before it is read again
            if (k + 1 >= I.ns) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __syncthreads();
            const int size = (int)(v >> 32);
            const int cum = cum_prev + size;
            if (!ok || cum >= I.n_stop || size == 0) {
                if (wv == 0) {
                    if (!ok || size == 0) atomicOr(&I.P.ctrl->status, ST_INTERNAL);
                    I.front_info[0] = k - 1;
                    I.front_info[1] = cum_prev;
                    I.front_info[2] = I.n_stop - cum_prev;
                    I.front_info[3] = k;
                    sh.own_cum[q] = -1;
                }
                continue;
            }
            if (wv == 0) {
                sh.own_cum[q] = cum;
                // clear the counters of front k + 1 (last read while waiting for
                // front k - 2); this chunk's own front-k publish, which front k + 1
                // waits for, is ordered after these stores
                if (lane <= PEEL_SHARDS) store_relaxed(&peel_slot(I.P.facc, k + 1)[lane * PEEL_STRIDE], 0ull);
            }
            if (k == 1) peel_transpose(I, c, sh);
            peel_chunk(I, k, c, sh);
            active = 1;
        }
        __syncthreads();
        if (!active) break;
    }
}

hipError_t launch_prepare(const HostPlan &hp, const BatchView &bv, hipStream_t s) {
    NSGA3_LAUNCH("init", k_init, dim3(hp.B), dim3(256), 0, s, bv);
    NSGA3_LAUNCH("prep", k_prep, dim3((hp.npt + hp.nref) / 256), dim3(256), 0, s, bv, hp.npt);
    return hipGetLastError();
}

hipError_t launch_nd_sort(const HostPlan &hp, const BatchView &bv, hipStream_t s) {
    for (int g = 0; g < hp.ngroups; ++g) {
        const int gs = hp.grp_start[g], gn = hp.grp_start[g + 1] - gs;
        const long long item0 = hp.grp_dom[g], n_items = hp.grp_dom[g + 1] - item0;
        const unsigned blocks = (unsigned)((n_items + 3) / 4);
#define NSGA3_DOM_CASE(MO)                                                                       \
    case MO:                                                                                     \
        NSGA3_LAUNCH("dominance", k_dominance<MO>, dim3(blocks), dim3(256), 0, s, bv, gs, gn,   \
                     item0, n_items);                                                            \
        break;
        switch (hp.grp_m[g]) {
            NSGA3_DOM_CASE(2) NSGA3_DOM_CASE(3) NSGA3_DOM_CASE(4) NSGA3_DOM_CASE(5)
            NSGA3_DOM_CASE(6) NSGA3_DOM_CASE(7) NSGA3_DOM_CASE(8) NSGA3_DOM_CASE(9)
            NSGA3_DOM_CASE(10) NSGA3_DOM_CASE(11) NSGA3_DOM_CASE(12) NSGA3_DOM_CASE(13)
            NSGA3_DOM_CASE(14) NSGA3_DOM_CASE(15) NSGA3_DOM_CASE(16)
            default: return hipErrorInvalidValue;
        }
#undef NSGA3_DOM_CASE
    }
    const int cap = 3 * device_info().cus;
    const int peel_blocks = hp.nchunk < cap ? hp.nchunk : cap;
    NSGA3_LAUNCH("peel", k_peel, dim3(peel_blocks), dim3(64 * PEEL_WAVES), 0, s, bv, hp.nchunk);
    return hipGetLastError();
}

}  // namespace nsga3
