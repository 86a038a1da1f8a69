// Quality indicators of a population, on the device: the inverted
// generational distance (IGD, the indicator of the paper's population-size
// study, Sec. IV) against points of a known optimal front, and the
// hypervolume (HV) in the paper's normalized form (Appendix E: reference
// point 1.01 f_max, ideal point 0.9 f_min, HV / HV_max with HV_max the
// volume of the box between them), estimated by counting dominated sample
// points of that box. Not part of the selection: they measure what a served
// run produced.
//
// Kernels:
//   k_igd_min   per front point r, the least squared distance to a
//               population point: 64 front points in the lanes, a slice of
//               the population through the scalar cache, slices merged by
//               an atomic min on the (non-negative) float bits
//   k_igd_sum   mean of the distances in a fixed order (deterministic)
//   k_hv_count  one sample point of the box per lane; counts the samples
//               that some population point weakly dominates
#include "nsga3_internal.h"

namespace nsga3 {

constexpr int IGD_SLICE = 256;  // population points per work item

__global__ __launch_bounds__(256) void k_igd_min(const float *F, int n, int m, const float *R,
                                                  int nr, unsigned *dmin, int nslice) {
    const long long item = uniform((long long)blockIdx.x * 4 + (threadIdx.x >> 6));
    const int rb = (int)(item / nslice), sl = (int)(item % nslice);
    const int r = rb * 64 + lane_id();
    if (rb * 64 >= nr) return;
    const bool in = r < nr;
    float y[NARROW_M];
#pragma unroll
    for (int k = 0; k < NARROW_M; ++k) y[k] = in && k < m ? R[(size_t)r * m + k] : 0.0f;
    const NSGA3_RO float *P = (const NSGA3_RO float *)F;
    const int p0 = sl * IGD_SLICE, p1 = min(p0 + IGD_SLICE, n);
    float best = INFINITY;
    for (int p = p0; p < p1; ++p) {
        float d2 = 0.0f;
#pragma unroll
        for (int k = 0; k < NARROW_M; ++k) {
            if (k < m) {
                const float diff = y[k] - P[(size_t)p * m + k];
                d2 = fmaf(diff, diff, d2);
            }
        }
        best = fminf(best, d2);
    }
    if (in && p0 < p1) atomicMin(&dmin[r], __float_as_uint(best));
}

__global__ __launch_bounds__(256) void k_igd_sum(const unsigned *dmin, int nr, double *out) {
    __shared__ double part[256];
    double s = 0.0;
    for (int r = threadIdx.x; r < nr; r += 256) s += (double)sqrtf(__uint_as_float(dmin[r]));
    part[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = part[0] / (double)nr;
}

// The box of the hypervolume estimate: sample i, objective k is
//   u = (sm64(seed ^ sm64(i << 8 | k)) >> 40) * 2^-24        (exact in FP32)
//   y_k = ideal_k + u * (ref_k - ideal_k)
// with each FP32 operation rounded on its own (no fused multiply-add), so a
// CPU that rounds the same operations in FP32 gets the same sample points.
struct HvBox {
    float ideal[NARROW_M];
    float ref[NARROW_M];
};

__global__ __launch_bounds__(256) void k_hv_count(const float *F, int n, int m, HvBox box,
                                                   long long samples, u64 seed,
                                                   unsigned long long *count) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    const bool valid = i < samples;
    float y[NARROW_M];
#pragma unroll
    for (int k = 0; k < NARROW_M; ++k) {
        y[k] = 0.0f;
        if (k < m) {
            const u64 h = sm64(seed ^ sm64(((u64)i << 8) | (u64)k));
            const float u = (float)(unsigned)(h >> 40) * 0x1p-24f;
            const float span = __fsub_rn(box.ref[k], box.ideal[k]);
            y[k] = __fadd_rn(box.ideal[k], __fmul_rn(u, span));
        }
    }
    const NSGA3_RO float *P = (const NSGA3_RO float *)F;
    bool covered = !valid;
    for (int p = 0; p < n; ++p) {
        bool dom = true;
#pragma unroll
        for (int k = 0; k < NARROW_M; ++k)
            if (k < m) dom = dom && P[(size_t)p * m + k] <= y[k];
        covered = covered || dom;
        if (ballot(!covered) == 0) break;  // every sample of the wave is dominated
    }
    const u64 hit = ballot(valid && covered);
    if (lane_id() == 0 && hit) atomicAdd(count, (unsigned long long)__popcll(hit));
}

// Zeroes the count, or sets every least squared distance to +inf.
__global__ __launch_bounds__(256) void k_fill_u32(unsigned *p, int n, unsigned v) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace nsga3

using namespace nsga3;

static bool al4(const void *p) { return ((uintptr_t)p & 3u) == 0; }

extern "C" {

size_t nsga3_igd_workspace_bytes(int32_t nr) {
    if (nr < 1 || nr > NSGA3_MAX_POINTS) return 0;
    return ((size_t)nr * 4 + 255) & ~(size_t)255;
}

int nsga3_igd(const float *F, int32_t n, int32_t m, const float *R, int32_t nr, double *igd,
              void *ws, size_t ws_bytes, void *stream) {
    if (!F || !R || !igd || !ws || n < 1 || n > NSGA3_MAX_POINTS || nr < 1 ||
        nr > NSGA3_MAX_POINTS || m < 2 || m > NARROW_M || !al4(F) || !al4(R) ||
        ((uintptr_t)igd & 7u) || ((uintptr_t)ws & 255u))
        return NSGA3_EINVAL;
    if (ws_bytes < nsga3_igd_workspace_bytes(nr)) return NSGA3_EWORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    unsigned *dmin = (unsigned *)ws;
    const int nslice = (n + IGD_SLICE - 1) / IGD_SLICE;
    const long long items = (long long)((nr + 63) / 64) * nslice;
    NSGA3_LAUNCH("igd_fill", k_fill_u32, dim3((nr + 255) / 256), dim3(256), 0, s, dmin, nr,
                 0x7f800000u);
    NSGA3_LAUNCH("igd_min", k_igd_min, dim3((unsigned)((items + 3) / 4)), dim3(256), 0, s, F, n, m,
                 R, nr, dmin, nslice);
    NSGA3_LAUNCH("igd_sum", k_igd_sum, dim3(1), dim3(256), 0, s, dmin, nr, igd);
    return hipGetLastError() == hipSuccess ? NSGA3_OK : NSGA3_EHIP;
}

int nsga3_hv_count(const float *F, int32_t n, int32_t m, const float *ideal, const float *ref,
                   int64_t samples, uint64_t seed, unsigned long long *count, void *stream) {
    if (!F || !ideal || !ref || !count || n < 1 || n > NSGA3_MAX_POINTS || m < 2 ||
        m > NARROW_M || samples < 1 || samples > ((int64_t)1 << 31) || !al4(F) ||
        ((uintptr_t)count & 7u))
        return NSGA3_EINVAL;
    HvBox box;
    for (int k = 0; k < NARROW_M; ++k) {
        box.ideal[k] = k < m ? ideal[k] : 0.0f;
        box.ref[k] = k < m ? ref[k] : 0.0f;
        if (k < m && !(box.ideal[k] <= box.ref[k])) return NSGA3_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    NSGA3_LAUNCH("hv_zero", k_fill_u32, dim3(1), dim3(256), 0, s, (unsigned *)count, 2, 0u);
    NSGA3_LAUNCH("hv_count", k_hv_count, dim3((unsigned)((samples + 255) / 256)), dim3(256), 0, s,
                 F, n, m, box, (long long)samples, seed, count);
    return hipGetLastError() == hipSuccess ? NSGA3_OK : NSGA3_EHIP;
}

}  // extern "C"
