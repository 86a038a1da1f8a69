// Internal declarations of libnsga3: the per-instance descriptor and batch
// view that every kernel reads, the device control block, device helpers
// shared by the kernels, and the host-side launchers.
//
// Every kernel works on a batch of independent selection instances (a plain
// call is a batch of one). Each instance has its own workspace region and a
// descriptor with absolute device pointers; the descriptors and the prefix
// arrays that map a global work index to (instance, local index) live in the
// batch header region of the workspace, written there by a copy kernel whose
// arguments carry the bytes (so a whole call is kernel launches only, and can
// be captured in a HIP graph).
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

// Which stages a call runs (selects the resets and the optional fusions).
enum : int {
    RUN_ND = 1,
    RUN_NORM = 2,
    RUN_ASSOC = 4,
    RUN_NICHE = 8,
    RUN_SELECT = 15,
    RUN_CACHE_TENSOR = 16,  // niche stage: the paper's cache-tensor loop instead of the closed form
};

// Objective counts up to NARROW_M run kernels specialized per m (values of
// one point in registers); larger m runs general kernels.
constexpr int NARROW_M = 16;

// Device-resident control block at the start of every instance's workspace.
struct Ctrl {
    int status;
    int list_count;          // length of the S_t index list
    unsigned zmin_enc[NSGA3_MAX_OBJECTIVES];   // ideal point, order-preserving encoding
    unsigned fmax_enc[NSGA3_MAX_OBJECTIVES];   // largest objective over S_t, same encoding
    u64 ext_key[NSGA3_MAX_OBJECTIVES];         // (ASF bits << 32) | index, min-reduced
    float zf[NSGA3_MAX_OBJECTIVES];            // ideal point
    float recip[NSGA3_MAX_OBJECTIVES];         // 1 / intercept, float32
    int lstar;               // water-fill level L*
    int rpick;               // picks made at level L*
    int all_pick;            // 1 if the whole last front is taken
    int fl_total;            // |F_l|
    int front_info[4];       // front_info of nsga3_select (stage calls use the caller's)
    float ideal_out[NSGA3_MAX_OBJECTIVES];
    double icpt_out[NSGA3_MAX_OBJECTIVES];
    int ext_out[NSGA3_MAX_OBJECTIVES];
    int degen_out;
    int ext_done;            // blocks of the extreme search that finished
};

// front ring of the peel: PEEL_RING slots, each with two tagged words per
// chunk, padded to whole 128-byte lines
constexpr int PEEL_RING = 4;
constexpr int front_slot_words(int W) { return (2 * W + 15) & ~15; }
constexpr int PT_ALIGN = 256;    // per-instance point and reference ranges are padded to this
constexpr int COMPACT_TILE = 256;  // points per compaction tile (one workgroup)
constexpr int TICKET_SHARDS = 32;   // peel chunk-claim counters of a batch
constexpr int TICKET_STRIDE = 32;   // u64 words between them (256 bytes)
constexpr int PLACE_BUCKETS = 1024;  // first-objective buckets of the point placement
constexpr int PLACE_RANK_BITS = 20;  // place key: bucket << PLACE_RANK_BITS | rank in bucket
static_assert(NSGA3_MAX_POINTS <= (1 << PLACE_RANK_BITS), "ranks in a bucket fit the key");
constexpr int PEEL_PIPE_GROUPS = 8; // most m-groups whose peels run one per group
                                    // (word g of each shard counts group g)

// Byte offsets of one instance's workspace regions (all 256-byte aligned).
struct Layout {
    int M, m, H, N, Mp, W, Hp;
    size_t ctrl, ft, nd, mask, ring, perm, pkey, bcount, row_ord, col_end, list, fn, rank, pi,
        dist, akey, wn, rho, cnt, off, fill, tpick, members, qrow, picked, tcnt, remain, emat,
        total;
};

Layout make_layout(int M, int m, int H, int N);

struct Ptrs {
    Ctrl *ctrl;
    float *ft;
    int *nd;
    u64 *mask;
    u64 *ring;          // peel front ring (tagged members per front)
    // Point placement (dominance and peel work on positions, not indices):
    int *perm;          // point at each position
    unsigned *pkey;     // per point: bucket << PLACE_RANK_BITS | rank within the bucket
    unsigned *bcount;   // points per bucket (PLACE_BUCKETS)
    int *row_ord;       // per row block jb: tiles (ib, jb) with ib < row_ord[jb] are ordered
    int *col_end;       // per column block c: its words from row block col_end[c] on are zero
    int *list;
    float *fn;
    int *rank, *pi;
    float *dist;
    u64 *akey;
    float *wn;
    int *rho, *cnt, *off, *fill, *tpick, *members, *picked;
    int *qrow;          // cache-tensor baseline: candidates of each reference in pick order
    int *tcnt;          // selected points per compaction tile
    u64 *remain;
    double *emat;       // m > NARROW_M: the intercept system [m][m], rhs, column maxima, b
};

Ptrs carve(const Layout &L, void *ws);

// One instance as the kernels see it.
struct Inst {
    const float *F;
    const float *Z;
    int *rank;          // in/out ranks
    int *front_info;    // in/out {l, |S|, K, l + 1}
    float *Fn;          // normalized objectives
    int *pi;
    float *dist;
    int *selected;
    float *ideal;
    double *intercept;
    int *extreme;
    int *degenerate;
    Ptrs P;
    u64 seed;
    int M, m, H, N, Mp, W, Hp;
    int n_stop;
    int G;              // dominance: triangle tiles per work item
    int R, nslice;      // association: references per slice, slices
};

// Descriptor memory (the batch header) is written by a call's first kernels
// and only read by every later kernel of the call. Reads through this
// address space are invariant loads, which the compiler may keep in
// registers or repeat across barriers, fences and atomics.
#define NSGA3_RO __attribute__((address_space(4)))
typedef const NSGA3_RO Inst CInst;

// Global index ranges: instance b owns [pref[b], pref[b+1]) of each kind.
// Point and reference ranges are padded to PT_ALIGN so that no 256-thread
// block straddles two instances. dom_pref / asc_pref run over `order`
// (instances sorted by m) and count per-wave work items; chunk_pref runs
// over `order` too, so that the chunks of one m-group are contiguous.
struct BatchView {
    CInst *tab;
    const NSGA3_RO int *pt_pref;
    const NSGA3_RO int *ref_pref;
    const NSGA3_RO int *chunk_pref;
    const NSGA3_RO int *order;
    const NSGA3_RO long long *dom_pref;
    const NSGA3_RO long long *asc_pref;
    u64 *ticket;        // peel chunk-claim counters (TICKET_SHARDS x TICKET_STRIDE words)
    int B;
    int run;            // RUN_* flags of this call
};

// ------------------------------------------------------------ device helpers

// Largest b in [0, n) with pref[b] <= x (pref[0] <= x < pref[n]).
template <typename T>
__device__ __forceinline__ int find_range(const NSGA3_RO T *pref, int n, T x) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pref[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

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

// Workgroup barrier that orders LDS accesses only: unlike __syncthreads it
// does not wait for this wave's global stores to complete.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Wave reductions by DPP moves (no LDS round trips). They follow the
// pattern of wave_incl_scan below: row shifts by 1, 2, 4, 8, then the row
// broadcasts of lanes 15 and 31; lanes without a source take the operation's
// identity, and lane 63 ends with the reduction over all 64 lanes, which is
// then read back into every lane. All lanes must be active.
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned dpp_u32(unsigned identity, unsigned v) {
    return (unsigned)__builtin_amdgcn_update_dpp((int)identity, (int)v, CTRL, ROWS, 0xf, false);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ u64 dpp_u64(u64 identity, u64 v) {
    const unsigned lo = dpp_u32<CTRL, ROWS>((unsigned)identity, (unsigned)v);
    const unsigned hi = dpp_u32<CTRL, ROWS>((unsigned)(identity >> 32), (unsigned)(v >> 32));
    return ((u64)hi << 32) | lo;
}

__device__ __forceinline__ u64 lane63_u64(u64 v) {
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)v, 63);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)(v >> 32), 63);
    return ((u64)hi << 32) | lo;
}

#define NSGA3_DPP_STEPS(STEP) \
    STEP(0x111, 0xf) STEP(0x112, 0xf) STEP(0x114, 0xf) STEP(0x118, 0xf) STEP(0x142, 0xa) STEP(0x143, 0xc)

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit integers");
    if constexpr (sizeof(T) == 4) {
        unsigned u = (unsigned)v;
#define NSGA3_STEP(C, R) u += dpp_u32<C, R>(0u, u);
        NSGA3_DPP_STEPS(NSGA3_STEP)
#undef NSGA3_STEP
        return (T)__builtin_amdgcn_readlane(u, 63);
    } else {
        u64 u = (u64)v;
#define NSGA3_STEP(C, R) u += dpp_u64<C, R>(0ull, u);
        NSGA3_DPP_STEPS(NSGA3_STEP)
#undef NSGA3_STEP
        return (T)lane63_u64(u);
    }
}

__device__ __forceinline__ u64 wave_min_u64(u64 v) {
#define NSGA3_STEP(C, R) { const u64 o = dpp_u64<C, R>(~0ull, v); v = o < v ? o : v; }
    NSGA3_DPP_STEPS(NSGA3_STEP)
#undef NSGA3_STEP
    return lane63_u64(v);
}

__device__ __forceinline__ u64 wave_max_u64(u64 v) {
#define NSGA3_STEP(C, R) { const u64 o = dpp_u64<C, R>(0ull, v); v = o > v ? o : v; }
    NSGA3_DPP_STEPS(NSGA3_STEP)
#undef NSGA3_STEP
    return lane63_u64(v);
}

__device__ __forceinline__ unsigned wave_min_u32(unsigned v) {
#define NSGA3_STEP(C, R) v = min(v, dpp_u32<C, R>(0xffffffffu, v));
    NSGA3_DPP_STEPS(NSGA3_STEP)
#undef NSGA3_STEP
    return __builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
#define NSGA3_STEP(C, R) v = max(v, dpp_u32<C, R>(0u, v));
    NSGA3_DPP_STEPS(NSGA3_STEP)
#undef NSGA3_STEP
    return __builtin_amdgcn_readlane(v, 63);
}

// Inclusive prefix sum over the 64 lanes of a wave.
// Inclusive scan over the 64 lanes with DPP moves (no LDS round trips):
// shifts by 1, 2, 4, 8 within each row of 16 lanes, then the last lane of
// row 0 (2) is added to row 1 (3), then lane 31 to rows 2 and 3. Lanes
// whose source lies outside the pattern, or whose row is masked off, add 0.
__device__ __forceinline__ int wave_incl_scan(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15, rows 1 and 3
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31, rows 2 and 3
    return v;
}

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

// (instance, local index) of a thread of a point- or reference-parallel
// kernel with 256-thread blocks over ranges padded to PT_ALIGN.
struct Local {
    int b;      // instance
    int i;      // local index of this thread
};
__device__ __forceinline__ Local locate(const NSGA3_RO int *pref, int B) {
    const int base = uniform((int)(blockIdx.x * blockDim.x));
    const int b = uniform(find_range(pref, B, base));
    return Local{b, base - pref[b] + (int)threadIdx.x};
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

// Per-instance start of a call (one workgroup, thread t): status, list
// counter, front fill default, normalization accumulators.
__device__ __forceinline__ void init_instance(Ctrl *ctrl, int *front_info, int n_stop, int run,
                                              unsigned *bcount, int t) {
    if (t == 0) {
        ctrl->status = 0;
        ctrl->list_count = 0;
        ctrl->ext_done = 0;
        if (run & RUN_ND) {
            // a defined value even if the peel stops on an internal error
            front_info[0] = 0;
            front_info[1] = 0;
            front_info[2] = n_stop;
            front_info[3] = 0;
        }
    }
    for (int k = t; k < NSGA3_MAX_OBJECTIVES; k += 256) {
        ctrl->zmin_enc[k] = 0xffffffffu;
        ctrl->fmax_enc[k] = 0u;
        ctrl->ext_key[k] = ~0ull;
    }
    if (run & RUN_ND) {
        static_assert(PLACE_BUCKETS == 4 * 256, "four bucket counts per thread");
#pragma unroll
        for (int q = 0; q < 4; ++q) bcount[t + 256 * q] = 0;  // placement counts
    }
}

// -------------------------------------------------------------- launchers

struct Dev {
    int cus;  // compute units of the current device
};
Dev device_info();

// Host-side plan of one call: totals and the m-groups of the batch.
struct HostPlan {
    int B;
    int npt, nref, nchunk;
    int ngroups;
    int grp_m[NSGA3_MAX_OBJECTIVES + 1];
    int grp_start[NSGA3_MAX_OBJECTIVES + 2];       // range of `order` per group
    long long grp_dom[NSGA3_MAX_OBJECTIVES + 2];   // dominance items before each group
    long long grp_asc[NSGA3_MAX_OBJECTIVES + 2];   // association items before each group
    int grp_chunk[NSGA3_MAX_OBJECTIVES + 2];       // 64-point chunks before each group
    int grp_max_W[NSGA3_MAX_OBJECTIVES + 1];       // widest instance of each group
    int max_W;
};

// Copies `bytes` host bytes to device memory `dst` with kernels whose
// arguments carry the data (graph-capturable; the host buffer may be reused
// as soon as the call returns). `bytes` is a multiple of 4.
hipError_t upload(const void *src, size_t bytes, void *dst, hipStream_t s);

// Generation step of served populations (descriptor table in ws).
size_t evolve_header_bytes(int B);
hipError_t launch_evolve(const nsga3_evolve_slot *slots, int B, char *ws, hipStream_t s);

// init_done: the instance was initialized with the header copy (k_blob_init).
hipError_t launch_prepare(const HostPlan &hp, const BatchView &bv, bool init_done, hipStream_t s);
// *through: in: the normalization and association sweeps may be pipelined
// with the peel (a whole selection whose groups all have m <= NARROW_M);
// out: they were (launch_normalize is then skipped and launch_associate only
// finishes).
hipError_t launch_nd_sort(const HostPlan &hp, const BatchView &bv, hipStream_t s, bool *through);
hipError_t launch_normalize(const HostPlan &hp, const BatchView &bv, hipStream_t s);
// sweeps_done: the per-group sweeps already ran (pipelined with the peel).
hipError_t launch_associate(const HostPlan &hp, const BatchView &bv, hipStream_t s,
                            bool sweeps_done);
void launch_norm_fused_group(const HostPlan &hp, const BatchView &bv, int g, hipStream_t s);
void launch_associate_group(const HostPlan &hp, const BatchView &bv, int g, hipStream_t s);
hipError_t launch_niche(const HostPlan &hp, const BatchView &bv, hipStream_t s);

// One-workgroup selection of a small instance (tiny.hip): whether the shape
// qualifies, and the launch (I: the planned descriptor of the instance).
bool tiny_fits(int M, int m, int H);
hipError_t launch_select_tiny(const Inst &I, hipStream_t s);

// dominance work items of an instance (waves): block row jb holds
// floor(jb / G) + 1 items of up to G column tiles each
long long dominance_tiles(int W);  // 64x64 tiles of the triangle ib <= jb

}  // namespace nsga3
