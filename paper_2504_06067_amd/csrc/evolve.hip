// Offspring generation around the selection (Sec. II-C: a mating pool and
// the variation operators SBX and polynomial mutation produce n offspring;
// Algorithm 1, "Crossover+Mutation"), with a synthetic objective map, for a
// batch of resident populations. This is the generation step that a served
// run repeats between selections; it is not part of the selection itself.
//
// Per slot (one population of N decision vectors in [0, 1)^d, m objectives):
//   init        rows 0..N-1 of X_new: x_ij uniform in [0, 1); F_new = f(x)
//   population  rows 0..N-1: the population, row r = X_old[sel[r]] (sel
//               NULL: row r of X_old), with its objectives
//   generation  population rows as above, then N offspring in rows N..2N-1:
//               pair k = i / 2 mates parents a, b drawn uniformly from the
//               population; child i % 2 of SBX (distribution index 20, every
//               variable crossed) then polynomial mutation (rate 1/d,
//               distribution index 20); values are clamped to [0, 1 - 2^-24]
// Objective map: y = A (x_1..x_{d-1} - 1/2), u = |y| / ||y|| (1/sqrt(m) each
// when y = 0), g = -0.3 ln(1 - x_d), f = u (1 + g). At a uniform x the radius
// 1 + g is 1 + Exponential(mean 0.3), the law of the large plain workload, and
// the optimal front is the positive unit sphere.
//
// Random numbers: h(seed, g, tag, i, j) = sm64(seed ^ sm64(tag << 58 |
// (g mod 2^16) << 42 | j << 32 | i)) with sm64 the SplitMix64 output function;
// a uniform in [0, 1) is (h >> 40) * 2^-24; an index below n is h mod n.
// Every draw depends only on (seed, generation, individual, variable), so a
// population evolves identically alone or batched with others.
#include <vector>

#include "nsga3_internal.h"

namespace nsga3 {

enum : unsigned {
    TAG_INIT = 4,
    TAG_PA = 5,
    TAG_PB = 6,
    TAG_SBX = 7,
    TAG_PM_APPLY = 8,
    TAG_PM_U = 9,
};

constexpr float EVO_ETA_C = 20.0f;
constexpr float EVO_ETA_M = 20.0f;
constexpr float EVO_XMAX = 0.99999994f;  // 1 - 2^-24
constexpr int EVO_NARROW_D = 64;         // widest d of the row-per-thread kernel

__device__ __forceinline__ u64 evo_hash(u64 seed, unsigned g, unsigned tag, unsigned i,
                                        unsigned j) {
    const u64 c = ((u64)tag << 58) | ((u64)(g & 0xffffu) << 42) | ((u64)(j & 0x3ffu) << 32) |
                  (u64)i;
    return sm64(seed ^ sm64(c));
}

__device__ __forceinline__ float evo_u01(u64 h) { return (float)(h >> 40) * 5.9604644775390625e-8f; }

__device__ __forceinline__ float clamp01(float x) { return fminf(fmaxf(x, 0.0f), EVO_XMAX); }

struct EvoSlot {
    const float *X_old;
    const int *sel;
    const float *F_old;
    float *X_new;
    float *F_new;
    const float *A;
    u64 seed;
    int N, d, m, g, mode, rows;
};

struct EvoView {
    const NSGA3_RO EvoSlot *slot;
    const NSGA3_RO int *row_pref;
    int B;
};

// Objectives of decision vector x (row of X_new just written by this thread).
__device__ __forceinline__ void evo_objectives(const NSGA3_RO EvoSlot &S, const float *x, float *f) {
    const int d = S.d, m = S.m;
    float y[NSGA3_MAX_EVOLVE_OBJECTIVES];
    for (int k = 0; k < m; ++k) y[k] = 0.0f;
    for (int j = 0; j + 1 < d; ++j) {
        const float c = x[j] - 0.5f;
        for (int k = 0; k < m; ++k) y[k] = fmaf(S.A[k * (d - 1) + j], c, y[k]);
    }
    float n2 = 0.0f;
    for (int k = 0; k < m; ++k) n2 = fmaf(y[k], y[k], n2);
    const float rad = 1.0f - 0.3f * logf(1.0f - x[d - 1]);
    if (n2 > 0.0f) {
        const float inv = 1.0f / sqrtf(n2);
        for (int k = 0; k < m; ++k) f[k] = fabsf(y[k]) * inv * rad;
    } else {
        const float u = 1.0f / sqrtf((float)m);
        for (int k = 0; k < m; ++k) f[k] = u * rad;
    }
}

__device__ __forceinline__ float sbx_beta(float u) {
    const float e = 1.0f / (EVO_ETA_C + 1.0f);
    return u <= 0.5f ? powf(2.0f * u, e) : powf(1.0f / (2.0f * (1.0f - u)), e);
}

__device__ __forceinline__ float pm_delta(float u) {
    const float e = 1.0f / (EVO_ETA_M + 1.0f);
    return u < 0.5f ? powf(2.0f * u, e) - 1.0f : 1.0f - powf(2.0f * (1.0f - u), e);
}

// One thread per output row of every slot with d <= EVO_NARROW_D.
__global__ __launch_bounds__(256) void k_evolve(EvoView ev) {
    const int base = uniform((int)(blockIdx.x * blockDim.x));
    const int b = uniform(find_range(ev.row_pref, ev.B, base));
    const NSGA3_RO EvoSlot &S = ev.slot[b];
    const int r = base - ev.row_pref[b] + (int)threadIdx.x;
    if (r >= S.rows || S.d > EVO_NARROW_D) return;
    const int N = S.N, d = S.d, m = S.m;
    float *xo = S.X_new + (size_t)r * d;
    float *fo = S.F_new + (size_t)r * m;
    if (S.mode == NSGA3_EVOLVE_INIT) {
        for (int j = 0; j < d; ++j) xo[j] = evo_u01(evo_hash(S.seed, 0u, TAG_INIT, (unsigned)r, (unsigned)j));
        float f[NSGA3_MAX_EVOLVE_OBJECTIVES];
        evo_objectives(S, xo, f);
        for (int k = 0; k < m; ++k) fo[k] = f[k];
        return;
    }
    if (r < N) {
        const int src = S.sel ? S.sel[r] : r;
        for (int j = 0; j < d; ++j) xo[j] = S.X_old[(size_t)src * d + j];
        for (int k = 0; k < m; ++k) fo[k] = S.F_old[(size_t)src * m + k];
        return;
    }
    const int i = r - N;
    const unsigned k2 = (unsigned)(i >> 1);
    const unsigned g = (unsigned)S.g;
    const int pa = (int)(evo_hash(S.seed, g, TAG_PA, k2, 0u) % (u64)N);
    const int pb = (int)(evo_hash(S.seed, g, TAG_PB, k2, 0u) % (u64)N);
    const int ra = S.sel ? S.sel[pa] : pa;
    const int rb = S.sel ? S.sel[pb] : pb;
    const float pm_rate = 1.0f / (float)d;
    for (int j = 0; j < d; ++j) {
        const float x1 = S.X_old[(size_t)ra * d + j];
        const float x2 = S.X_old[(size_t)rb * d + j];
        const float beta = sbx_beta(evo_u01(evo_hash(S.seed, g, TAG_SBX, k2, (unsigned)j)));
        float y = (i & 1) ? 0.5f * ((1.0f - beta) * x1 + (1.0f + beta) * x2)
                          : 0.5f * ((1.0f + beta) * x1 + (1.0f - beta) * x2);
        y = clamp01(y);
        if (evo_u01(evo_hash(S.seed, g, TAG_PM_APPLY, (unsigned)i, (unsigned)j)) < pm_rate)
            y = clamp01(y + pm_delta(evo_u01(evo_hash(S.seed, g, TAG_PM_U, (unsigned)i, (unsigned)j))));
        xo[j] = y;
    }
    float f[NSGA3_MAX_EVOLVE_OBJECTIVES];
    evo_objectives(S, xo, f);
    for (int k = 0; k < m; ++k) fo[k] = f[k];
}

// Float sum over the 64 lanes of a wave (butterfly; every lane gets it).
__device__ __forceinline__ float wave_fsum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Wide decision vectors (d > EVO_NARROW_D): one wave per output row, lanes
// over the variables (coalesced rows), the same per-variable operations and
// random draws as k_evolve; the objective map's sums over the variables are
// per-lane partial sums reduced across the wave. Grid: 4 rows per block over
// every slot's padded row range; rows of narrow slots leave at once.

__global__ __launch_bounds__(256) void k_evolve_wide(EvoView ev) {
    const int base = uniform((int)(blockIdx.x * 4));
    const int b = uniform(find_range(ev.row_pref, ev.B, base));
    const NSGA3_RO EvoSlot &S = ev.slot[b];
    const int r = base - ev.row_pref[b] + (int)(threadIdx.x >> 6);
    if (r >= S.rows || S.d <= EVO_NARROW_D) return;  // wave-uniform
    const int lane = lane_id();
    const int N = S.N, d = S.d, m = S.m;
    float *xo = S.X_new + (size_t)r * d;
    float *fo = S.F_new + (size_t)r * m;
    if (S.mode != NSGA3_EVOLVE_INIT && r < N) {
        const int src = S.sel ? S.sel[r] : r;
        for (int j = lane; j < d; j += 64) xo[j] = S.X_old[(size_t)src * d + j];
        if (lane < m) fo[lane] = S.F_old[(size_t)src * m + lane];
        return;
    }
    const int i = r - N;
    const unsigned k2 = (unsigned)(i >> 1);
    const unsigned g = (unsigned)S.g;
    int ra = 0, rb = 0;
    if (S.mode != NSGA3_EVOLVE_INIT) {
        const int pa = (int)(evo_hash(S.seed, g, TAG_PA, k2, 0u) % (u64)N);
        const int pb = (int)(evo_hash(S.seed, g, TAG_PB, k2, 0u) % (u64)N);
        ra = S.sel ? S.sel[pa] : pa;
        rb = S.sel ? S.sel[pb] : pb;
    }
    const float pm_rate = 1.0f / (float)d;
    float y[NSGA3_MAX_EVOLVE_OBJECTIVES];
    for (int k = 0; k < m; ++k) y[k] = 0.0f;
    float xlast = 0.0f;
    for (int j = lane; j < d; j += 64) {
        float x;
        if (S.mode == NSGA3_EVOLVE_INIT) {
            x = evo_u01(evo_hash(S.seed, 0u, TAG_INIT, (unsigned)r, (unsigned)j));
        } else {
            const float x1 = S.X_old[(size_t)ra * d + j];
            const float x2 = S.X_old[(size_t)rb * d + j];
            const float beta = sbx_beta(evo_u01(evo_hash(S.seed, g, TAG_SBX, k2, (unsigned)j)));
            x = (i & 1) ? 0.5f * ((1.0f - beta) * x1 + (1.0f + beta) * x2)
                        : 0.5f * ((1.0f + beta) * x1 + (1.0f - beta) * x2);
            x = clamp01(x);
            if (evo_u01(evo_hash(S.seed, g, TAG_PM_APPLY, (unsigned)i, (unsigned)j)) < pm_rate)
                x = clamp01(x + pm_delta(evo_u01(evo_hash(S.seed, g, TAG_PM_U, (unsigned)i, (unsigned)j))));
        }
        xo[j] = x;
        if (j + 1 < d) {
            const float c = x - 0.5f;
            for (int k = 0; k < m; ++k) y[k] = fmaf(S.A[k * (d - 1) + j], c, y[k]);
        } else {
            xlast = x;
        }
    }
    float n2 = 0.0f;
    for (int k = 0; k < m; ++k) {
        y[k] = wave_fsum(y[k]);
        n2 = fmaf(y[k], y[k], n2);
    }
    const float xl = __uint_as_float(
        __builtin_amdgcn_readlane(__float_as_uint(xlast), (d - 1) & 63));
    const float rad = 1.0f - 0.3f * logf(1.0f - xl);
    const float inv = n2 > 0.0f ? 1.0f / sqrtf(n2) : 0.0f;
    const float u0 = 1.0f / sqrtf((float)m);
    for (int k = 0; k < m; ++k)
        if (lane == k) fo[k] = (n2 > 0.0f ? fabsf(y[k]) * inv : u0) * rad;
}

size_t evolve_header_bytes(int B) {
    const size_t a = ((size_t)B * sizeof(EvoSlot) + 255) & ~(size_t)255;
    return a + (((size_t)(B + 1) * 4 + 255) & ~(size_t)255);
}

hipError_t launch_evolve(const nsga3_evolve_slot *slots, int B, char *ws, hipStream_t s) {
    std::vector<unsigned char> hdr(evolve_header_bytes(B), 0);
    const size_t off_pref = ((size_t)B * sizeof(EvoSlot) + 255) & ~(size_t)255;
    EvoSlot *tab = (EvoSlot *)hdr.data();
    int *pref = (int *)(hdr.data() + off_pref);
    pref[0] = 0;
    for (int b = 0; b < B; ++b) {
        const nsga3_evolve_slot &q = slots[b];
        EvoSlot e;
        e.X_old = q.X_old;
        e.sel = q.sel;
        e.F_old = q.F_old;
        e.X_new = q.X_new;
        e.F_new = q.F_new;
        e.A = q.A;
        e.seed = q.seed;
        e.N = q.N;
        e.d = q.d;
        e.m = q.m;
        e.g = q.generation;
        e.mode = q.mode;
        e.rows = q.mode == NSGA3_EVOLVE_GENERATION ? 2 * q.N : q.N;
        tab[b] = e;
        pref[b + 1] = pref[b] + (e.rows + PT_ALIGN - 1) / PT_ALIGN * PT_ALIGN;
    }
    hipError_t e = upload(hdr.data(), hdr.size(), ws, s);
    if (e != hipSuccess) return e;
    EvoView ev;
    ev.slot = (const NSGA3_RO EvoSlot *)ws;
    ev.row_pref = (const NSGA3_RO int *)(ws + off_pref);
    ev.B = B;
    bool narrow = false, wide = false;
    for (int b = 0; b < B; ++b) (slots[b].d > EVO_NARROW_D ? wide : narrow) = true;
    if (narrow)
        NSGA3_LAUNCH("evolve", k_evolve, dim3((unsigned)(pref[B] / 256)), dim3(256), 0, s, ev);
    if (wide)
        NSGA3_LAUNCH("evolve", k_evolve_wide, dim3((unsigned)(pref[B] / 4)), dim3(256), 0, s, ev);
    return hipGetLastError();
}

}  // namespace nsga3
