// Association (paper Sec. II-C: each solution goes to the reference point of
// least perpendicular distance; Eq. 1, read as ||f|| sin(theta), the true
// perpendicular distance; Algorithm 2: argmin and min over the reference axis).
//
// The distance tensor of the paper (2N x H) is never materialized: a wave
// holds 64 points of S_t in its lanes and sweeps a slice of the unit
// reference directions, read through the scalar cache from a
// structure-of-arrays copy. The distance is formed from the explicit
// residual r = f - (f . w) w, whose FP32 rounding error scales with ||f||
// rather than with the (possibly tiny) distance. Slices are merged with a
// 64-bit atomic min on (d^2 bits << 32 | j): least distance, then least j.
//
// Kernels:
//   k_assoc_init   resets the S_t list counter
//   k_assoc_prep   unit reference directions (SoA), validity check of Z,
//                  S_t list, key init, pi = dist = -1 outside S_t
//   k_associate    the fused sweep
//   k_assoc_final  pi and dist from the merged keys
#include "nsga3_internal.h"

namespace nsga3 {

__global__ void k_assoc_init(Ctrl *ctrl, bool reset_status) {
    if (threadIdx.x == 0) {
        if (reset_status) ctrl->status = 0;
        ctrl->list_count = 0;
    }
}

__global__ __launch_bounds__(256) void k_assoc_prep(const float *__restrict__ Z, int H, int Hp,
                                                     int m, float *__restrict__ wn,
                                                     const int *__restrict__ rank,
                                                     const int *__restrict__ front_info, int M,
                                                     int *__restrict__ list,
                                                     u64 *__restrict__ akey, int *pi, float *dist,
                                                     Ctrl *ctrl) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    // unit reference directions, padded refs repeat the last real one
    bool bad = false;
    if (t < Hp) {
        const int j = t < H ? t : H - 1;
        float s = 0.0f;
        for (int k = 0; k < m; ++k) {
            const float v = Z[(size_t)j * m + k];
            bad |= !(v >= 0.0f) || !isfinite(v);
            s = fmaf(v, v, s);
        }
        bad |= !(s > 0.0f);
        const float inv = bad ? 0.0f : 1.0f / sqrtf(s);
        for (int k = 0; k < m; ++k) wn[(size_t)k * Hp + t] = Z[(size_t)j * m + k] * inv;
    }
    if (ballot(bad) != 0 && lane_id() == 0) atomicOr(&ctrl->status, ST_BADREF);
    // S_t list
    const int l = front_info[0];
    const bool in = t < M && rank[t] >= 0 && rank[t] <= l;
    if (t < M && !in) {
        pi[t] = -1;
        dist[t] = -1.0f;
    }
    const u64 bal = ballot(in);
    if (bal == 0) return;
    int base = 0;
    if (lane_id() == 0) base = atomicAdd(&ctrl->list_count, __popcll(bal));
    base = __shfl(base, 0, 64);
    if (in) {
        list[base + mbcnt(bal)] = t;
        akey[t] = ~0ull;
    }
}

// Work item = (block of 64 list entries, slice of R references). Grid covers
// the largest possible S_t; items past the actual list length exit at once.
// The reference loop reads the unit directions through the scalar cache
// (the item is wave-uniform) and is unrolled by four.
template <int MO>
__device__ __forceinline__ void assoc_ref(const float (&f)[MO], const float *__restrict__ wn,
                                          int Hp, int j, float &best, int &bj) {
    float w[MO];
#pragma unroll
    for (int k = 0; k < MO; ++k) w[k] = wn[(size_t)k * Hp + j];
    float p = f[0] * w[0];
#pragma unroll
    for (int k = 1; k < MO; ++k) p = fmaf(f[k], w[k], p);
    float d2 = 0.0f;
#pragma unroll
    for (int k = 0; k < MO; ++k) {
        const float r = fmaf(-p, w[k], f[k]);
        d2 = fmaf(r, r, d2);
    }
    if (d2 < best) { best = d2; bj = j; }
}

template <int MO>
__global__ __launch_bounds__(256) void k_associate(const float *__restrict__ Fn,
                                                    const int *__restrict__ list,
                                                    const float *__restrict__ wn, int H, int Hp,
                                                    int R, int nslice, u64 *__restrict__ akey,
                                                    const Ctrl *__restrict__ ctrl) {
    const int n = ctrl->list_count;
    const long long item = uniform((long long)blockIdx.x * 4 + (threadIdx.x >> 6));
    const int pb = (int)(item / nslice);
    const int sl = (int)(item % nslice);
    if (pb * 64 >= n) return;
    const int i = pb * 64 + lane_id();
    const bool in = i < n;
    const int x = in ? list[i] : list[pb * 64];
    float f[MO];
#pragma unroll
    for (int k = 0; k < MO; ++k) f[k] = Fn[(size_t)x * MO + k];
    const int h0 = sl * R;
    const int h1 = min(h0 + R, H);
    float best = INFINITY;
    int bj = h0;
    int j = h0;
    for (; j + 4 <= h1; j += 4) {
        assoc_ref<MO>(f, wn, Hp, j, best, bj);
        assoc_ref<MO>(f, wn, Hp, j + 1, best, bj);
        assoc_ref<MO>(f, wn, Hp, j + 2, best, bj);
        assoc_ref<MO>(f, wn, Hp, j + 3, best, bj);
    }
    for (; j < h1; ++j) assoc_ref<MO>(f, wn, Hp, j, best, bj);
    if (in && h0 < h1) {
        const u64 key = ((u64)__float_as_uint(best) << 32) | (unsigned)bj;
        atomicMin(&akey[x], key);
    }
}

__global__ __launch_bounds__(256) void k_assoc_final(const int *__restrict__ list,
                                                      const u64 *__restrict__ akey, int H,
                                                      int *pi, float *dist, Ctrl *ctrl) {
    const int n = ctrl->list_count;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int x = list[i];
    const u64 key = akey[x];
    int j = (int)(unsigned)(key & 0xffffffffull);
    if (j < 0 || j >= H) {
        atomicOr(&ctrl->status, ST_INTERNAL);
        j = 0;
    }
    pi[x] = j;
    dist[x] = sqrtf(__uint_as_float((unsigned)(key >> 32)));
}

hipError_t launch_associate(const Layout &L, const Ptrs &P, const float *Fn, const int *rank,
                            const int *front_info, const float *Z, int *pi, float *dist,
                            bool reset_status, hipStream_t s) {
    const int M = L.M, m = L.m, H = L.H, Hp = L.Hp;
    NSGA3_LAUNCH("assoc_init", k_assoc_init, dim3(1), dim3(64), 0, s, P.ctrl, reset_status);
    const int nt = M > Hp ? M : Hp;
    NSGA3_LAUNCH("assoc_prep", k_assoc_prep, dim3((nt + 255) / 256), dim3(256), 0, s, Z, H, Hp, m, P.wn,
                       rank, front_info, M, P.list, P.akey, pi, dist, P.ctrl);
    // slice the references so that the grid holds about 16k waves
    const long long pblocks = (M + 63) / 64;
    long long R = (long long)H * pblocks / 16384;
    R = ((R + 15) / 16) * 16;
    if (R < 32) R = 32;
    if (R > H) R = H;
    const int nslice = (int)((H + R - 1) / R);
    const long long items = pblocks * nslice;
    const unsigned blocks = (unsigned)((items + 3) / 4);
#define NSGA3_ASSOC_CASE(MO)                                                                  \
    case MO:                                                                                  \
        NSGA3_LAUNCH("associate", k_associate<MO>, dim3(blocks), dim3(256), 0, s, Fn, P.list, P.wn, \
                           H, Hp, (int)R, nslice, P.akey, P.ctrl);                            \
        break;
    switch (m) {
        NSGA3_ASSOC_CASE(2) NSGA3_ASSOC_CASE(3) NSGA3_ASSOC_CASE(4) NSGA3_ASSOC_CASE(5)
        NSGA3_ASSOC_CASE(6) NSGA3_ASSOC_CASE(7) NSGA3_ASSOC_CASE(8) NSGA3_ASSOC_CASE(9)
        NSGA3_ASSOC_CASE(10) NSGA3_ASSOC_CASE(11) NSGA3_ASSOC_CASE(12) NSGA3_ASSOC_CASE(13)
        NSGA3_ASSOC_CASE(14) NSGA3_ASSOC_CASE(15) NSGA3_ASSOC_CASE(16)
        default: return hipErrorInvalidValue;
    }
#undef NSGA3_ASSOC_CASE
    NSGA3_LAUNCH("assoc_final", k_assoc_final, dim3((M + 255) / 256), dim3(256), 0, s, P.list, P.akey, H,
                       pi, dist, P.ctrl);
    return hipGetLastError();
}

}  // namespace nsga3
