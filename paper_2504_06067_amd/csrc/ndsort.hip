// Non-dominated sorting (paper Sec. II-C; Algorithm 1 "Non-dominated-sort")
// as a bit-packed dominance matrix followed by front peeling.
//
// Dominance matrix layout ("word-major"): mask[w * Mp + j] is a 64-bit word
// whose bit b is set iff point 64*w + b dominates point j. A wave of 64
// consecutive j therefore reads or writes 512 contiguous bytes.
//
// Kernels:
//   k_nd_init    reset of the control block
//   k_nd_prep    SoA copy of the objectives (+inf padding), finiteness check,
//                zeroed dominator counts, alive set of front 0
//   k_dominance  triangle of 64x64 tiles; per tile both directions from one
//                set of 2m compares per pair; fused dominator counts
//   k_peel       fronts peeled by a ticketed work queue: items of front k
//                wait until every item of front k-1 completed
#include "nsga3_internal.h"

namespace nsga3 {

__global__ void k_nd_init(Ctrl *ctrl, int *fcum, int *front_info, int n_stop, bool reset_status) {
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
        fcum[0] = 0;
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
            ft[(size_t)k * Mp + j] = v;
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

// Lane `lane` of the result takes the wave-uniform value v; other lanes keep old.
__device__ __forceinline__ unsigned write_lane(unsigned old, unsigned v, int lane) {
    return lane_id() == lane ? v : old;
}

// Number of work items for block rows 0..jb-1 when row jb holds floor(jb/G)+1
// items of up to G column tiles each.
__device__ __forceinline__ long long items_before(long long jb, long long G) {
    long long q = jb / G, s = jb % G;
    return jb + G * q * (q - 1) / 2 + q * s;
}

// One wave per work item: the 64 points of block row jb sit in the lanes
// (as the dominated side j); the item sweeps up to G column blocks ib <= jb.
// For every i of block ib (uniform, read through the scalar cache) the wave
// forms lt = {j : f_i < f_j in some objective} and gt = {j : f_i > f_j in
// some objective} with 2m compares; then
//   i dominates j  <=>  j in lt \ gt   (shifted into lane j's word A)
//   j dominates i  <=>  j in gt \ lt   (the whole mask is row i's word B).
template <int MO>
__global__ __launch_bounds__(256) void k_dominance(const float *__restrict__ ft, int Mp, int W,
                                                    int G, long long n_items,
                                                    u64 *__restrict__ mask,
                                                    int *__restrict__ nd) {
    const int lane = lane_id();
    const long long item = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
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
    for (int k = 0; k < MO; ++k) fj[k] = ft[(size_t)k * Mp + jglob];

    int cnt_j = 0;
    for (int ib = ib0; ib < ib1; ++ib) {
        const float *fi = ft + (size_t)ib * 64;
        unsigned a_lo = 0, a_hi = 0, b_lo = 0, b_hi = 0;
#pragma unroll
        for (int r = 63; r >= 0; --r) {
            u64 lt = 0, gt = 0;
#pragma unroll
            for (int k = 0; k < MO; ++k) {
                const float v = fi[(size_t)k * Mp + r];
                lt |= ballot(v < fj[k]);
                gt |= ballot(v > fj[k]);
            }
            const u64 i_dom_j = lt & ~gt;
            const u64 j_dom_i = gt & ~lt;
            const unsigned bit = (unsigned)(i_dom_j >> lane) & 1u;
            if (r >= 32) a_hi = (a_hi << 1) | bit;
            else a_lo = (a_lo << 1) | bit;
            b_lo = write_lane(b_lo, (unsigned)j_dom_i, r);
            b_hi = write_lane(b_hi, (unsigned)(j_dom_i >> 32), r);
        }
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
constexpr int PEEL_UNROLL = 8;

// Front peeling. Work item t covers front k = t / W and the 64 points of
// chunk c = t % W. Items are taken in ticket order, so an item waits only for
// items with smaller tickets, which are held by running workgroups: the wait
// always ends. Front 0 is {j : no dominator} from the fused counts. For k > 0,
// a point j alive at front k belongs to it iff no alive point dominates it,
// i.e. (mask[w][j] & alive_k[w]) == 0 for every word w. The alive sets of
// consecutive fronts alternate between two bitsets. The peel stops once the
// fronts ranked so far hold at least n_stop points.
//
// Control flow is wave-uniform everywhere around the workgroup barriers:
// wave 0 takes tickets and waits with all its lanes (atomics contribute only
// from lane 0), so no loop of this kernel can split a wave's lanes between
// iterations.
__global__ __launch_bounds__(1024) void k_peel(const u64 *__restrict__ mask,
                                                const int *__restrict__ nd, int M, int Mp, int W,
                                                int n_stop, u64 *alive, int *rank, int *fcum,
                                                Ctrl *ctrl, int *front_info) {
    __shared__ u64 s_ticket;
    __shared__ int s_exit;
    __shared__ u64 s_hit;
    const int lane = lane_id();
    const int wv = uniform((int)(threadIdx.x >> 6));
    const u64 C = (u64)W;
    const u64 one = lane == 0 ? 1ull : 0ull;
    // Safety bounds (never reached by a correct run): a block processes at most
    // (fronts + 1) * W <= (M + 2) * W items, and no wait lasts 2^26 polls.
    const u64 max_items = (u64)(M + 2) * C;
    u64 done_items = 0;

    for (;;) {
        if (wv == 0) {
            const u64 t = uniform(atomicAdd(&ctrl->ticket, one));
            const u64 k = t / C;
            int ex = 0;
            if (++done_items > max_items) {
                atomicOr(&ctrl->status, ST_INTERNAL);
                atomicExch(&ctrl->finished, 1u);
                ex = 1;
            } else if (k > 0) {
                const u64 target = k * C;
                for (unsigned polls = 0;; ++polls) {
                    if (uniform(load_acquire(&ctrl->completed)) >= target) break;
                    if (uniform((int)load_acquire(&ctrl->finished))) { ex = 1; break; }
                    if (polls == (1u << 26)) {
                        atomicOr(&ctrl->status, ST_INTERNAL);
                        atomicExch(&ctrl->finished, 1u);
                        ex = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
                if (!ex) {
                    const int cum = uniform(load_acquire(&ctrl->ranked));  // fronts 0..k-1
                    const int prev = uniform(fcum[k - 1]);                // fronts 0..k-2
                    if (cum >= n_stop || cum == prev) {
                        if (cum == prev) atomicOr(&ctrl->status, ST_INTERNAL);
                        front_info[0] = (int)k - 1;
                        front_info[1] = prev;
                        front_info[2] = n_stop - prev;
                        front_info[3] = (int)k;
                        __threadfence();
                        atomicExch(&ctrl->finished, 1u);
                        ex = 1;
                    } else {
                        fcum[k] = cum;
                    }
                }
            }
            s_ticket = t;
            s_exit = ex;
            s_hit = 0;
        }
        __syncthreads();
        if (uniform(s_exit)) break;
        __threadfence();
        const u64 t = uniform(s_ticket);
        const int k = (int)(t / C);
        const int c = (int)(t % C);
        const u64 *alive_k = alive + (size_t)(k & 1) * W;
        u64 *alive_n = alive + (size_t)((k + 1) & 1) * W;
        const u64 aw = uniform(alive_k[c]);
        const int j = c * 64 + lane;
        u64 newly;
        if (k == 0) {
            newly = aw & ballot(nd[j] == 0);
        } else {
            if (aw != 0) {
                bool hit = false;
                for (int w0 = wv; w0 < W; w0 += PEEL_WAVES * PEEL_UNROLL) {
                    u64 a[PEEL_UNROLL], x[PEEL_UNROLL];
#pragma unroll
                    for (int u = 0; u < PEEL_UNROLL; ++u) {
                        const int w = w0 + u * PEEL_WAVES;
                        a[u] = (w < W) ? alive_k[w] : 0ull;
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
            if ((newly >> lane) & 1ull) rank[j] = k;
            alive_n[c] = aw & ~newly;
        }
        __threadfence();
        __syncthreads();
        if (wv == 0) {
            atomicAdd(&ctrl->ranked, lane == 0 ? __popcll(newly) : 0);
            __threadfence();
            atomicAdd(&ctrl->completed, one);
        }
    }
}

hipError_t launch_nd_sort(const Layout &L, const Ptrs &P, const float *F, int n_stop, int *rank,
                          int *front_info, bool reset_status, hipStream_t s) {
    const int M = L.M, m = L.m, Mp = L.Mp, W = L.W;
    hipLaunchKernelGGL(k_nd_init, dim3(1), dim3(64), 0, s, P.ctrl, P.fcum, front_info, n_stop,
                       reset_status);
    hipLaunchKernelGGL(k_nd_prep, dim3((Mp + 255) / 256), dim3(256), 0, s, F, M, m, Mp, P.ft,
                       P.nd, rank, P.alive, P.ctrl);
    const int G = 8;
    long long n_items = (long long)W + (long long)G * ((W / G) * (long long)(W / G - 1) / 2) +
                        (long long)(W / G) * (W % G);
    const unsigned blocks = (unsigned)((n_items + 3) / 4);
#define NSGA3_DOM_CASE(MO)                                                                   \
    case MO:                                                                                 \
        hipLaunchKernelGGL(k_dominance<MO>, dim3(blocks), dim3(256), 0, s, P.ft, Mp, W, G,  \
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
    hipLaunchKernelGGL(k_peel, dim3(peel_blocks), dim3(64 * PEEL_WAVES), 0, s, P.mask, P.nd, M,
                       Mp, W, n_stop, P.alive, rank, P.fcum, P.ctrl, front_info);
    return hipGetLastError();
}

}  // namespace nsga3
