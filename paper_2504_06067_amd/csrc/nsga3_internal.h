// Internal declarations of libnsga3: workspace layout, the device control
// block, device helpers shared by the kernels, and the host-side launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/nsga3.h"

namespace nsga3 {

typedef unsigned long long u64;

// Status bits accumulated in Ctrl::status; nsga3_read_status maps them to the
// public codes (non-finite first, then invalid reference, then internal).
enum : int {
    ST_NONFINITE = 1,
    ST_BADREF = 2,
    ST_INTERNAL = 4,
};

// Device-resident control block at offset 0 of every workspace.
struct Ctrl {
    int status;
    int front_info[4];      // {l, |S|, K, fronts}: written by the peel
    u64 ticket;             // peel work-queue tickets
    u64 completed;          // peel items completed
    int ranked;             // points ranked so far
    unsigned finished;      // peel finished flag
    int list_count;         // length of the S_t index list
    unsigned zmin_enc[NSGA3_MAX_OBJECTIVES];   // ideal point, order-preserving encoding
    unsigned fmax_enc[NSGA3_MAX_OBJECTIVES];   // largest objective over S_t, same encoding
    u64 ext_key[NSGA3_MAX_OBJECTIVES];         // (ASF bits << 32) | index, min-reduced
    float zf[NSGA3_MAX_OBJECTIVES];            // ideal point
    float recip[NSGA3_MAX_OBJECTIVES];         // 1 / intercept, float32
    int lstar;              // water-fill level L*
    int rpick;              // picks made at level L*
    int all_pick;           // 1 if the whole last front is taken
    int fl_total;           // |F_l|
    // normalization outputs of nsga3_select (the stage call writes the caller's)
    float ideal_out[NSGA3_MAX_OBJECTIVES];
    double icpt_out[NSGA3_MAX_OBJECTIVES];
    int ext_out[NSGA3_MAX_OBJECTIVES];
    int degen_out;
};

// Byte offsets of every workspace region (all 256-byte aligned).
struct Layout {
    int M, m, H, N, Mp, W, Hp, ns;
    size_t ctrl, ft, nd, mask, rowm, wit, alive, facc, list, fn, rank, pi, dist, akey, wn,
        rho, cnt, off, fill, tpick, members, picked, remain, tiles, total;
};

Layout make_layout(int M, int m, int H, int N);

struct Ptrs {
    Ctrl *ctrl;
    float *ft;
    int *nd;
    u64 *mask;
    u64 *rowm;
    int *wit;
    u64 *alive;
    int *list;
    u64 *facc;
    float *fn;
    int *rank, *pi;
    float *dist;
    u64 *akey;
    float *wn;
    int *rho, *cnt, *off, *fill, *tpick, *members, *picked;
    u64 *remain;
    int *tiles;
};

Ptrs carve(const Layout &L, void *ws);

// ------------------------------------------------------------ device helpers

__device__ __forceinline__ u64 sm64(u64 x) {
    u64 z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ u64 tie_key(u64 seed, unsigned tag, unsigned j, unsigned L) {
    u64 packed = ((u64)tag << 62) | ((u64)L << 32) | (u64)j;
    return sm64(seed ^ sm64(packed));
}

// Monotone map float -> uint32 (for atomic min/max on floats without NaN).
__device__ __forceinline__ unsigned f2ord(float f) {
    unsigned u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float ord2f(unsigned u) {
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Number of set bits of `mask` below this lane.
__device__ __forceinline__ int mbcnt(u64 mask) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0));
}

__device__ __forceinline__ u64 ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Values read from LDS are divergent to the compiler even when every lane
// reads the same word. Loops and branches that contain workgroup barriers must
// be driven by provably uniform values, so such reads go through these.
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ u64 uniform(u64 v) {
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
    return ((u64)hi << 32) | lo;
}
__device__ __forceinline__ long long uniform(long long v) { return (long long)uniform((u64)v); }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ u64 wave_min_u64(u64 v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        u64 w = __shfl_xor(v, o, 64);
        v = w < v ? w : v;
    }
    return v;
}

__device__ __forceinline__ u64 wave_max_u64(u64 v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        u64 w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    return v;
}

__device__ __forceinline__ unsigned wave_min_u32(unsigned v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, (unsigned)__shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, (unsigned)__shfl_xor(v, o, 64));
    return v;
}

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int w = __shfl_up(v, o, 64);
        if (lane >= o) v += w;
    }
    return v;
}

__device__ __forceinline__ unsigned load_acquire(const unsigned *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int load_acquire(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u64 load_acquire(const u64 *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------- instrumentation

// When profiling is enabled for a kernel name, a ProfScope around its launch
// records a pair of HIP events on the launch stream (events come from a pool
// created by nsga3_profile_enable; nothing is allocated at launch time).
struct ProfScope {
    int slot;
    hipStream_t stream;
    ProfScope(const char *name, hipStream_t s);
    ~ProfScope();
};

// Enqueue a kernel on stream `s` (which must be in scope), under a ProfScope
// named after the kernel.
#define NSGA3_LAUNCH(name, ...)              \
    do {                                     \
        ::nsga3::ProfScope ps_(name, s);     \
        hipLaunchKernelGGL(__VA_ARGS__);     \
    } while (0)

// -------------------------------------------------------------- launchers

struct Dev {
    int cus;  // compute units of the current device
};
Dev device_info();

// non-dominated sort
hipError_t launch_nd_sort(const Layout &L, const Ptrs &P, const float *F, int n_stop,
                          int *rank, int *front_info, bool reset_status, hipStream_t s);
// normalization
hipError_t launch_normalize(const Layout &L, const Ptrs &P, const float *F, const int *rank,
                            const int *front_info, float *Fn, float *ideal, double *intercept,
                            int *extreme, int *degenerate, bool reset_status, hipStream_t s);
// association
hipError_t launch_associate(const Layout &L, const Ptrs &P, const float *Fn, const int *rank,
                            const int *front_info, const float *Z, int *pi, float *dist,
                            bool reset_status, hipStream_t s);
// niching
hipError_t launch_niche(const Layout &L, const Ptrs &P, const int *rank, const int *front_info,
                        const int *pi, const float *dist, u64 seed, int *selected,
                        bool reset_status, hipStream_t s);

}  // namespace nsga3
