// Non-dominated sorting (paper Sec. II-C; Algorithm 1 "Non-dominated-sort")
// as a bit-packed dominance matrix followed by front peeling.
//
// Dominance matrix layout ("word-major"): mask[w * Mp + j] is a 64-bit word
// whose bit b is set iff point 64*w + b dominates point j. A wave of 64
// consecutive j therefore reads or writes 512 contiguous bytes.
//
// Kernels:
//   k_nd_init    reset of the control block
//   k_nd_prep    tile-major copy of the objectives (64 points x m coordinates
//                contiguous per tile, +inf padding), finiteness check,
//                zeroed dominator counts, alive set of front 0
//   k_dominance  triangle of 64x64 tiles; per tile both directions from one
//                set of 2m compares per pair; fused dominator counts
//   k_peel       fronts peeled by a ticketed work queue: items of front k
//                wait until every item of front k-1 completed
#include <utility>

#include "nsga3_internal.h"

namespace nsga3 {

// front-peeling ring of completion counters: 3 slots of 32 shard counters and
// one top word, each on its own 256-byte line
constexpr int PEEL_SHARDS = 32;
constexpr int PEEL_STRIDE = 32;                       // u64 words between counters (256 B)
constexpr int PEEL_SLOT = (PEEL_SHARDS + 1) * PEEL_STRIDE;
constexpr int PEEL_OWN_CAP = 2048;

__global__ void k_nd_init(Ctrl *ctrl, u64 *ring, int *front_info, int n_stop, bool reset_status) {
    for (int i = threadIdx.x; i < 3 * PEEL_SLOT; i += blockDim.x) ring[i] = 0;
    if (threadIdx.x == 0) {
        if (reset_status) ctrl->status = 0;
        // a defined value even if the peel stops on an internal error
        front_info[0] = 0;
        front_info[1] = 0;
        front_info[2] = n_stop;
        front_info[3] = 0;
        ctrl->ticket = 0;
        ctrl->completed = 0;
        ctrl->ranked = 0;
        ctrl->finished = 0;
    }
}

__global__ __launch_bounds__(256) void k_nd_prep(const float *__restrict__ F, int M, int m, int Mp,
                                                  float *__restrict__ ft, int *__restrict__ nd,
                                                  int *__restrict__ rank, u64 *__restrict__ alive0,
                                                  Ctrl *ctrl) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    if (j < Mp) {
        for (int k = 0; k < m; ++k) {
            float v = INFINITY;
            if (j < M) {
                v = F[(size_t)j * m + k];
                bad |= !isfinite(v);
            }
            ft[((size_t)(j >> 6) * m + k) * 64 + (j & 63)] = v;
        }
        nd[j] = 0;
        if (j < M) rank[j] = NSGA3_UNRANKED;
        if ((j & 63) == 0) {
            int valid = M - j;
            alive0[j >> 6] = valid >= 64 ? ~0ull : (valid <= 0 ? 0ull : ((1ull << valid) - 1));
        }
    }
    if (ballot(bad) != 0 && lane_id() == 0) atomicOr(&ctrl->status, ST_NONFINITE);
}

// (a << 1) | bit(lane) for every lane, with the bits taken from a wave mask:
// one v_addc with the mask as carry-in (a + a + carry).
__device__ __forceinline__ unsigned shift_in(unsigned a, u64 mask) {
    unsigned r;
    u64 carry_out;
    asm("v_addc_co_u32 %0, %1, %2, %2, %3" : "=v"(r), "=s"(carry_out) : "v"(a), "s"(mask));
    return r;
}

// Lane R of `old` takes the wave-uniform value v.
template <int R>
__device__ __forceinline__ unsigned write_lane(unsigned old, unsigned v) {
    asm("v_writelane_b32 %0, %1, %2" : "+v"(old) : "s"(v), "i"(R));
    return old;
}

// Number of work items for block rows 0..jb-1 when row jb holds floor(jb/G)+1
// items of up to G column tiles each.
__device__ __forceinline__ long long items_before(long long jb, long long G) {
    long long q = jb / G, s = jb % G;
    return jb + G * q * (q - 1) / 2 + q * s;
}

// One compare step against column point i = 64 * ib + R (uniform): the wave
// masks lt = {j : f_i < f_j in some objective}, gt = {j : f_i > f_j in some
// objective} come from 2m compares; then
//   i dominates j  <=>  j in lt \ gt   (bit R of lane j's word A)
//   j dominates i  <=>  j in gt \ lt   (the whole mask is row i's word B)
template <int MO, int R>
__device__ __forceinline__ void dom_step(const float *__restrict__ fi, const float (&fj)[MO],
                                         unsigned &a_lo, unsigned &a_hi, unsigned &b_lo,
                                         unsigned &b_hi) {
    u64 lt = 0, gt = 0;
#pragma unroll
    for (int k = 0; k < MO; ++k) {
        const float v = fi[k * 64 + R];
        lt |= ballot(v < fj[k]);
        gt |= ballot(v > fj[k]);
    }
    const u64 i_dom_j = lt & ~gt;
    const u64 j_dom_i = gt & ~lt;
    if (R >= 32) a_hi = shift_in(a_hi, i_dom_j);
    else a_lo = shift_in(a_lo, i_dom_j);
    b_lo = write_lane<R>(b_lo, (unsigned)j_dom_i);
    b_hi = write_lane<R>(b_hi, (unsigned)(j_dom_i >> 32));
}

// R runs 63 down to 0 so that the shifted-in bit of point 64*ib + R lands at
// bit R (of the high word for R >= 32).
template <int MO, int... Is>
__device__ __forceinline__ void dom_tile(std::integer_sequence<int, Is...>,
                                         const float *__restrict__ fi, const float (&fj)[MO],
                                         unsigned &a_lo, unsigned &a_hi, unsigned &b_lo,
                                         unsigned &b_hi) {
    (dom_step<MO, 63 - Is>(fi, fj, a_lo, a_hi, b_lo, b_hi), ...);
}

// One wave per work item: the 64 points of block row jb sit in the lanes
// (as the dominated side j); the item sweeps up to G column blocks ib <= jb,
// reading the column points through the scalar cache.
template <int MO>
__global__ __launch_bounds__(256) void k_dominance(const float *__restrict__ ft, int Mp, int W,
                                                    int G, long long n_items,
                                                    u64 *__restrict__ mask,
                                                    int *__restrict__ nd) {
    const int lane = lane_id();
    const long long item = uniform((long long)blockIdx.x * 4 + (threadIdx.x >> 6));
    if (item >= n_items) return;
    // locate the block row: largest jb with items_before(jb) <= item
    int lo = 0, hi = W;  // items_before(lo) <= item < items_before(hi)
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (items_before(mid, G) <= item) lo = mid; else hi = mid;
    }
    const int jb = lo;
    const int g = (int)(item - items_before(jb, G));
    const int ib0 = g * G;
    const int ib1 = min(ib0 + G, jb + 1);

    const size_t jglob = (size_t)jb * 64 + lane;
    float fj[MO];
#pragma unroll
    for (int k = 0; k < MO; ++k) fj[k] = ft[((size_t)jb * MO + k) * 64 + lane];

    int cnt_j = 0;
    for (int ib = ib0; ib < ib1; ++ib) {
        unsigned a_lo = 0, a_hi = 0, b_lo = 0, b_hi = 0;
        const float *fi = (const float *)__builtin_assume_aligned(ft + (size_t)ib * MO * 64, 256);
        dom_tile<MO>(std::make_integer_sequence<int, 64>{}, fi, fj, a_lo, a_hi, b_lo, b_hi);
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

constexpr int PEEL_WAVES = 16;
constexpr int PEEL_UNROLL = 12;

__device__ __forceinline__ u64 load_relaxed(const u64 *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int load_relaxed(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_relaxed(u64 *p, u64 v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_relaxed(int *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Front peeling.
//
// Chunk c holds the 64 points 64c .. 64c+63. Front 0 is {j : no dominator}
// (fused counts of the dominance kernel). A point j alive at front k > 0
// belongs to it iff no alive point dominates it: (mask[w][j] & alive_k[w])
// == 0 for every word w. The alive sets of consecutive fronts alternate
// between two bitsets. The peel stops once the ranked fronts hold n_stop
// points.
//
// Scheduling. While ranking front 0, workgroups claim chunks from a ticket
// counter until every chunk is claimed; a workgroup then owns its chunks for
// all later fronts. Only running workgroups claim, and no workgroup waits
// before all chunks are claimed and ranked for front 0, so every wait ends.
// A workgroup records at most PEEL_OWN_CAP chunks; if every running
// workgroup were full the front-0 wait would time out into an error status.
//
// Completion. Per front, chunk c adds (points ranked << 32) + 1 to shard
// counter c % PEEL_SHARDS; the last chunk of a shard promotes the shard total
// into the front's top word, which the waiting workgroups poll. Counters live
// in a ring of three front slots; the slot of front k + 1 is cleared while
// front k is processed (after front k - 1 completed, nobody reads it).
//
// Memory ordering. Cross-workgroup words (alive bitsets, counters) are
// written and read only with agent-scope atomics, which go to the coherent
// level; each chunk waits for its coherent stores before its counter add, so
// a workgroup that sees a front complete reads the published alive words.
// No L2 write-back or invalidation is needed on this path.
//
// Control flow is wave-uniform around every workgroup barrier: wave 0 makes
// the scheduling decisions with all its lanes and shares them through LDS.

__device__ __forceinline__ u64 *peel_slot(u64 *ring, int k) { return ring + (size_t)(k % 3) * PEEL_SLOT; }

// Ranks the points of chunk c that are alive at front k and have no alive
// dominator; publishes the chunk's result. All 16 waves take part.
__device__ __forceinline__ void peel_chunk(const u64 *__restrict__ mask, const int *__restrict__ nd,
                                           int Mp, int W, int k, int c, u64 *alive, int *rank,
                                           u64 *ring, u64 &s_hit) {
    const int lane = lane_id();
    const int wv = uniform((int)(threadIdx.x >> 6));
    const u64 *alive_k = alive + (size_t)(k & 1) * W;
    u64 *alive_n = alive + (size_t)((k + 1) & 1) * W;
    const u64 aw = uniform(load_relaxed(&alive_k[c]));
    const int j = c * 64 + lane;
    u64 newly;
    if (k == 0) {
        newly = aw & ballot(nd[j] == 0);
    } else {
        __syncthreads();  // every wave has read s_hit of the previous chunk
        if (wv == 0) s_hit = 0;
        __syncthreads();
        if (aw != 0) {
            bool hit = false;
            for (int w0 = wv; w0 < W; w0 += PEEL_WAVES * PEEL_UNROLL) {
                u64 a[PEEL_UNROLL], x[PEEL_UNROLL];
#pragma unroll
                for (int u = 0; u < PEEL_UNROLL; ++u) {
                    const int w = w0 + u * PEEL_WAVES;
                    a[u] = (w < W) ? load_relaxed(&alive_k[w]) : 0ull;
                    x[u] = (w < W) ? mask[(size_t)w * Mp + j] : 0ull;
                }
#pragma unroll
                for (int u = 0; u < PEEL_UNROLL; ++u) hit |= (a[u] & x[u]) != 0;
                const u64 hb = ballot(hit) & aw;
                if (hb) atomicOr(&s_hit, hb);
                const u64 seen = uniform(__hip_atomic_load(&s_hit, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_WORKGROUP)) | hb;
                if (seen == aw) break;
            }
        }
        __syncthreads();
        newly = aw & ~uniform(s_hit);
    }
    if (wv == 0) {
        if ((newly >> lane) & 1ull) rank[j] = k;  // read only by later kernels
        store_relaxed(&alive_n[c], aw & ~newly);
        __builtin_amdgcn_s_waitcnt(0);
        u64 *slot = peel_slot(ring, k);
        const int sh = c % PEEL_SHARDS;
        const u64 add = ((u64)__popcll(newly) << 32) | 1ull;
        const u64 old = uniform(__hip_atomic_fetch_add(&slot[sh * PEEL_STRIDE], lane == 0 ? add : 0ull,
                                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        const unsigned shard_chunks = (unsigned)((W - sh + PEEL_SHARDS - 1) / PEEL_SHARDS);
        if ((unsigned)(old & 0xffffffffull) + 1u == shard_chunks) {
            // last chunk of this shard: promote the shard total
            const u64 total = (((old >> 32) + (u64)__popcll(newly)) << 32) | 1ull;
            __hip_atomic_fetch_add(&slot[PEEL_SHARDS * PEEL_STRIDE], lane == 0 ? total : 0ull,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

__global__ __launch_bounds__(1024) void k_peel(const u64 *__restrict__ mask,
                                                const int *__restrict__ nd, int M, int Mp, int W,
                                                int n_stop, u64 *alive, int *rank, u64 *ring,
                                                Ctrl *ctrl, int *front_info
#ifdef NSGA3_PEEL_TRACE
                                                , u64 *trace
#endif
                                                ) {
    __shared__ int s_own[PEEL_OWN_CAP];
    __shared__ u64 s_hit;
    __shared__ u64 s_val;
    __shared__ int s_flag;
    const int lane = lane_id();
    const int wv = uniform((int)(threadIdx.x >> 6));
    const u64 one = lane == 0 ? 1ull : 0ull;
    const unsigned shards_used = (unsigned)(W < PEEL_SHARDS ? W : PEEL_SHARDS);

    // front 0: claim and rank chunks until all are claimed
    int nown = 0;
    for (;;) {
        if (wv == 0) s_val = uniform(atomicAdd(&ctrl->ticket, one));
        __syncthreads();
        const u64 t = uniform(s_val);
        __syncthreads();
        if (t >= (u64)W) break;
        const int c = (int)t;
        peel_chunk(mask, nd, Mp, W, 0, c, alive, rank, ring, s_hit);
        if (wv == 0) s_own[nown] = c;
        ++nown;
        if (nown == PEEL_OWN_CAP) break;
    }
    __syncthreads();
    // a workgroup without chunks has nothing left to do; the owners of the
    // chunks report the front fill
    if (nown == 0) return;

    int cum = 0;
    for (int k = 1;; ++k) {
        // wait for front k - 1
        if (wv == 0) {
            const u64 *top = peel_slot(ring, k - 1) + PEEL_SHARDS * PEEL_STRIDE;
            u64 v = 0;
            int ok = 1;
            for (unsigned polls = 0;; ++polls) {
                v = uniform(load_relaxed(top));
                if ((unsigned)(v & 0xffffffffull) >= shards_used) break;
                if (polls == (1u << 26)) { ok = 0; break; }
                __builtin_amdgcn_s_sleep(2);
            }
            s_val = v;
            s_flag = ok;
        }
        __syncthreads();
        const u64 v = uniform(s_val);
        const int ok = uniform(s_flag);
        __syncthreads();
        const int size = (int)(v >> 32);
        const int prev = cum;
        cum += size;
        if (!ok || cum >= n_stop || size == 0) {
            if (wv == 0) {
                if (!ok || size == 0) atomicOr(&ctrl->status, ST_INTERNAL);
                front_info[0] = k - 1;
                front_info[1] = prev;
                front_info[2] = n_stop - prev;
                front_info[3] = k;
            }
            break;
        }
        // clear the counters of front k + 1 (last read while waiting for front k - 2);
        // this workgroup's own front-k publish, which front k + 1 waits for, is
        // ordered after these stores
        if (wv == 0 && lane <= PEEL_SHARDS) store_relaxed(&peel_slot(ring, k + 1)[lane * PEEL_STRIDE], 0ull);
        for (int q = 0; q < nown; ++q) {
            const int c = uniform(s_own[q]);
#ifdef NSGA3_PEEL_TRACE
            if (threadIdx.x == 0 && k < 16) trace[2 * (k * W + c)] = __builtin_amdgcn_s_memrealtime();
#endif
            peel_chunk(mask, nd, Mp, W, k, c, alive, rank, ring, s_hit);
#ifdef NSGA3_PEEL_TRACE
            if (threadIdx.x == 0 && k < 16) trace[2 * (k * W + c) + 1] = __builtin_amdgcn_s_memrealtime();
#endif
        }
    }
}

hipError_t launch_nd_sort(const Layout &L, const Ptrs &P, const float *F, int n_stop, int *rank,
                          int *front_info, bool reset_status, hipStream_t s) {
    const int M = L.M, m = L.m, Mp = L.Mp, W = L.W;
    NSGA3_LAUNCH("nd_init", k_nd_init, dim3(1), dim3(256), 0, s, P.ctrl, P.facc, front_info,
                 n_stop, reset_status);
    NSGA3_LAUNCH("nd_prep", k_nd_prep, dim3((Mp + 255) / 256), dim3(256), 0, s, F, M, m, Mp, P.ft,
                       P.nd, rank, P.alive, P.ctrl);
    const int G = 8;
    long long n_items = (long long)W + (long long)G * ((W / G) * (long long)(W / G - 1) / 2) +
                        (long long)(W / G) * (W % G);
    const unsigned blocks = (unsigned)((n_items + 3) / 4);
#define NSGA3_DOM_CASE(MO)                                                                   \
    case MO:                                                                                 \
        NSGA3_LAUNCH("dominance", k_dominance<MO>, dim3(blocks), dim3(256), 0, s, P.ft, Mp, W, G,  \
                           n_items, P.mask, P.nd);                                           \
        break;
    switch (m) {
        NSGA3_DOM_CASE(2) NSGA3_DOM_CASE(3) NSGA3_DOM_CASE(4) NSGA3_DOM_CASE(5)
        NSGA3_DOM_CASE(6) NSGA3_DOM_CASE(7) NSGA3_DOM_CASE(8) NSGA3_DOM_CASE(9)
        NSGA3_DOM_CASE(10) NSGA3_DOM_CASE(11) NSGA3_DOM_CASE(12) NSGA3_DOM_CASE(13)
        NSGA3_DOM_CASE(14) NSGA3_DOM_CASE(15) NSGA3_DOM_CASE(16)
        default: return hipErrorInvalidValue;
    }
#undef NSGA3_DOM_CASE
    const int peel_blocks = W < 2 * device_info().cus ? W : 2 * device_info().cus;
    NSGA3_LAUNCH("peel", k_peel, dim3(peel_blocks), dim3(64 * PEEL_WAVES), 0, s, P.mask, P.nd, M,
                 Mp, W, n_stop, P.alive, rank, P.facc, P.ctrl, front_info
#ifdef NSGA3_PEEL_TRACE
                 , P.akey
#endif
                 );
    return hipGetLastError();
}

}  // namespace nsga3
