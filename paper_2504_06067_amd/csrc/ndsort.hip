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
constexpr int ALIVE_PAD = 16;  // u64 words per alive word (one 128-byte line)

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
            alive0[(size_t)(j >> 6) * ALIVE_PAD] =
                valid >= 64 ? ~0ull : (valid <= 0 ? 0ull : ((1ull << valid) - 1));
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

constexpr int PEEL_WAVES = 8;
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
// belongs to it iff no alive point dominates it. Fronts after the first are
// found with witnesses: every alive point keeps one alive dominator (its
// witness) and is re-examined only once its witness has been ranked. The
// re-examination resumes the scan of j's row at the witness's word: the
// words before it held no alive dominator when they were scanned, and the
// alive set only shrinks. Over the whole peel each row is read about once.
// The scans read a row-major copy of the dominance matrix (row j = the W
// words of point j's dominators), which each workgroup writes for its own
// chunks when front 1 starts; when front 0 already fills N it is never built.
// The alive sets of consecutive fronts alternate between two bitsets.
//
// Scheduling. While ranking front 0, workgroups claim chunks from a ticket
// counter until every chunk is claimed; a workgroup then owns its chunks for
// all later fronts. Only running workgroups claim, and no workgroup waits
// before all chunks are claimed and ranked for front 0, so every wait ends.
// A workgroup records at most PEEL_OWN_CAP chunks; if every running
// workgroup were full the front-0 wait would time out into an error status.
//
// Completion. Per front, chunk c adds (points ranked << 32) + 1 to shard
// counter c % PEEL_SHARDS (a fire-and-forget atomic); a waiting workgroup
// reads the 32 shards with one wave and sums them. Counters live in a ring of
// three front slots; the slot of front k + 1 is cleared while front k is
// processed (after front k - 1 completed, nobody reads it).
//
// Memory ordering. Alive words and counters are written with agent-scope
// atomic stores, which go to the coherent level; each chunk waits for its
// stores before its counter add. A workgroup polls the counters with relaxed
// atomic loads, and once a front is complete issues one agent-scope acquire
// fence, after which ordinary cached loads see the published alive words.
// The row-major copy and the witnesses of a chunk are touched only by its
// owner. No L2 write-back is needed on this path.
//
// Control flow is wave-uniform around every workgroup barrier: wave 0 makes
// the scheduling decisions with all its lanes and shares them through LDS.
constexpr int PEEL_LDS_ALIVE = 2048;  // alive words staged in LDS (M <= 131072)

__device__ __forceinline__ u64 *peel_slot(u64 *ring, int k) { return ring + (size_t)(k % 3) * PEEL_SLOT; }

// Alive bitset of front k: slot k % ns of the alive ring; the word of chunk c
// sits alone on a 128-byte line (ALIVE_PAD words), so no two workgroups ever
// write the same line and a slot is never cached before it is read.
__device__ __forceinline__ u64 *alive_slot(u64 *aring, int W, int ns, int k) {
    return aring + (size_t)(k % ns) * W * ALIVE_PAD;
}

struct PeelShared {
    int own[PEEL_OWN_CAP];
    union {                    // the transpose (front 1 start) and the scans never overlap
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
__device__ void peel_transpose(const u64 *__restrict__ mask, u64 *__restrict__ rowm, int *wit,
                               int Mp, int W, int c, PeelShared &sh) {
    const int lane = lane_id();
    const int wv = uniform((int)(threadIdx.x >> 6));
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
    if (threadIdx.x < 64) wit[c * 64 + lane] = -1;
}

// Ranks the points of chunk c that are alive at front k and have no alive
// dominator; publishes the chunk's result. All 16 waves take part.
#ifdef NSGA3_PEEL_TRACE
__device__ u64 *g_trace;
#define PEEL_MARK(i)                                                                       \
    if (k == 2 && threadIdx.x == 0)                                                       \
        g_trace[2 * 16 * W + 8 * c + (i)] = __builtin_amdgcn_s_memrealtime();
#else
#define PEEL_MARK(i)
#endif
__device__ void peel_chunk(const int *__restrict__ nd, const u64 *__restrict__ rowm, int *wit,
                           int W, int ns, int k, int c, u64 *alive, int *rank, u64 *ring,
                           PeelShared &sh) {
    const int lane = lane_id();
    const int wv = uniform((int)(threadIdx.x >> 6));
    const u64 *alive_k = alive_slot(alive, W, ns, k);
    u64 *alive_n = alive_slot(alive, W, ns, k + 1);
    const u64 aw = uniform(alive_k[(size_t)c * ALIVE_PAD]);
    const int j = c * 64 + lane;
    u64 newly;
    if (k == 0) {
        newly = aw & ballot(nd[j] == 0);
    } else {
        const bool staged = W <= PEEL_LDS_ALIVE;
        PEEL_MARK(0)
        __syncthreads();  // the previous chunk is done with the shared words
        if (staged && aw != 0)
            for (int w = threadIdx.x; w < W; w += blockDim.x) sh.alive[w] = alive_k[(size_t)w * ALIVE_PAD];
        if (wv == 0) sh.newly = 0;
        __syncthreads();
        PEEL_MARK(1)
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
        PEEL_MARK(2)
        const u64 need = uniform(sh.need);
        const int nneed = __popcll(need);
        // wave wv re-examines the needing points wv, wv + PEEL_WAVES, ... (lane
        // order); the first 64-word round of all of them is issued at once
        constexpr int PER = 64 / PEEL_WAVES;
        int pl[PER], wpos[PER];
        u64 xr[PER];
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
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            xr[q] = 0;
            wpos[q] = 0;
            if (q < mine) {
                const int jp = c * 64 + pl[q];
                const int wp = uniform(wit[jp]);
                wpos[q] = wp < 0 ? 0 : (wp >> 6);
                const int w = wpos[q] + lane;
                if (w < W)
                    xr[q] = rowm[(size_t)jp * W + w] &
                            (staged ? sh.alive[w] : alive_k[(size_t)w * ALIVE_PAD]);
            }
        }
        for (int q = 0; q < mine; ++q) {
            const int p = pl[q];
            const int jp = c * 64 + p;
            const u64 *row = rowm + (size_t)jp * W;
            int found = -1;
            u64 x = xr[q];
            for (int pos = wpos[q];;) {
                const u64 b = ballot(x != 0);
                if (b) {
                    // new witness: among the alive dominators in the first word that
                    // has any, the one with the most dominators of its own (a proxy
                    // for the deepest, which stays alive longest)
                    const int L = __ffsll((long long)b) - 1;
                    const unsigned lo = __builtin_amdgcn_readlane((unsigned)x, L);
                    const unsigned hi = __builtin_amdgcn_readlane((unsigned)(x >> 32), L);
                    const u64 xl = ((u64)hi << 32) | lo;
                    const int cand = (pos + L) * 64 + lane;
                    const bool has = (xl >> lane) & 1ull;
                    const u64 key = has ? (((u64)(unsigned)nd[cand] << 32) | (unsigned)(~cand)) : 0ull;
                    const u64 best = wave_max_u64(key);
                    found = (int)~(unsigned)(best & 0xffffffffull);
                    break;
                }
                pos += 64;
                if (pos >= W) break;
                const int w = pos + lane;
                x = 0;
                if (w < W) x = row[w] & (staged ? sh.alive[w] : alive_k[(size_t)w * ALIVE_PAD]);
            }
            if (lane == 0) wit[jp] = found;
            if (found < 0 && lane == 0) atomicOr(&sh.newly, 1ull << p);
        }
        __syncthreads();
        PEEL_MARK(3)
        newly = aw & uniform(sh.newly);
    }
    if (wv == 0) {
        store_relaxed(&alive_n[(size_t)c * ALIVE_PAD], aw & ~newly);
        __builtin_amdgcn_s_waitcnt(0);
        u64 *slot = peel_slot(ring, k);
        const u64 add = ((u64)__popcll(newly) << 32) | 1ull;
        __hip_atomic_fetch_add(&slot[(c % PEEL_SHARDS) * PEEL_STRIDE], lane == 0 ? add : 0ull,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((newly >> lane) & 1ull) rank[j] = k;  // read only by later kernels
#ifdef NSGA3_PEEL_TRACE
        if (k == 2 && lane == 0) {
            g_trace[2 * 16 * W + 8 * c + 4] = __builtin_amdgcn_s_memrealtime();
            g_trace[2 * 16 * W + 8 * c + 5] = blockIdx.x;
            g_trace[2 * 16 * W + 8 * c + 6] = __popcll(uniform(sh.need));
        }
#endif
    }
}

__global__ __launch_bounds__(64 * PEEL_WAVES) void k_peel(const u64 *__restrict__ mask,
                                                const int *__restrict__ nd, int M, int Mp, int W,
                                                int n_stop, int ns, u64 *alive, int *rank,
                                                u64 *ring, u64 *rowm, int *wit, Ctrl *ctrl,
                                                int *front_info
#ifdef NSGA3_PEEL_TRACE
                                                , u64 *trace
#endif
                                                ) {
    __shared__ PeelShared sh;
#ifdef NSGA3_PEEL_TRACE
    g_trace = trace;
#endif
    // drop cached lines of alive slots read by an earlier call on this workspace
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const int lane = lane_id();
    const int wv = uniform((int)(threadIdx.x >> 6));
    const u64 one = lane == 0 ? 1ull : 0ull;

    // front 0: claim and rank chunks until all are claimed
    int nown = 0;
    for (;;) {
        if (wv == 0) sh.val = uniform(atomicAdd(&ctrl->ticket, one));
        __syncthreads();
        const u64 t = uniform(sh.val);
        __syncthreads();
        if (t >= (u64)W) break;
        const int c = (int)t;
        peel_chunk(nd, rowm, wit, W, ns, 0, c, alive, rank, ring, sh);
        if (wv == 0) sh.own[nown] = c;
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
            const u64 *slot = peel_slot(ring, k - 1);
            u64 v = 0;
            int ok = 1;
            for (unsigned polls = 0;; ++polls) {
                // lanes 0..31 read one shard each; the wave sums (count, size)
                u64 part = lane < PEEL_SHARDS ? load_relaxed(&slot[lane * PEEL_STRIDE]) : 0ull;
                v = uniform(wave_sum(part));
                if ((unsigned)(v & 0xffffffffull) >= (unsigned)W) break;
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
        if (k + 1 >= ns) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
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
        if (k == 1)
            for (int q = 0; q < nown; ++q) peel_transpose(mask, rowm, wit, Mp, W, uniform(sh.own[q]), sh);
        for (int q = 0; q < nown; ++q) {
            const int c = uniform(sh.own[q]);
#ifdef NSGA3_PEEL_TRACE
            if (threadIdx.x == 0 && k < 16) trace[2 * (k * W + c)] = __builtin_amdgcn_s_memrealtime();
#endif
            peel_chunk(nd, rowm, wit, W, ns, k, c, alive, rank, ring, sh);
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
    const int peel_blocks = W < 3 * device_info().cus ? W : 3 * device_info().cus;
    NSGA3_LAUNCH("peel", k_peel, dim3(peel_blocks), dim3(64 * PEEL_WAVES), 0, s, P.mask, P.nd, M,
                 Mp, W, n_stop, L.ns, P.alive, rank, P.facc, P.rowm, P.wit, P.ctrl, front_info
#ifdef NSGA3_PEEL_TRACE
                 , P.akey
#endif
                 );
    return hipGetLastError();
}

}  // namespace nsga3
