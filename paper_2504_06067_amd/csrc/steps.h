// Steps shared by the multi-kernel path and the one-workgroup path for
// small instances: the same floating-point operations in the same order, so
// both give bit-identical results.
#pragma once

#include "nsga3_internal.h"

namespace nsga3 {

// Doubles move between lanes as two 32-bit halves.
__device__ __forceinline__ double read_lane_f64(double v, int L) {
    const u64 u = (u64)__double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)u, L);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)(u >> 32), L);
    return __longlong_as_double((long long)(((u64)hi << 32) | lo));
}

// One wave per instance (I: the instance's descriptor, from the batch
// header or a kernel argument). E[k][j] =
// f(e_k)_j - z_j in FP64; E b = 1 is solved by Gaussian elimination with
// partial pivoting (largest |pivot|, least row on ties), the rows spread over
// the lanes (each row stays in its lane and carries its position; a swap
// exchanges two positions), every product and difference rounded separately;
// a_k = 1 / b_k
// unless degenerate.
// Sources: the encoded ideal point and maxima, the extreme keys and the
// objectives F [M][MO]; destinations zf (ideal point) and recip (1 / a) as
// float32, besides the instance's outputs. The multi-kernel path passes its
// control block; the one-workgroup path LDS copies.
template <int MO, typename InstT>
__device__ void norm_solve(InstT &I, const unsigned *zenc, const unsigned *fenc, const u64 *ekey,
                           const float *F, float *zf_out, float *recip_out) {
    Ctrl *ctrl = I.P.ctrl;
    const int lane = lane_id();
    const int M = I.M;
    // ideal point, extreme indices, per-objective span (lane k: objective k)
    int bad = 0;
    double zk = 0.0, fmxk = 0.0;
    int ek = 0;
    if (lane < MO) {
        const float zf = ord2f(zenc[lane]);
        zk = (double)zf;
        fmxk = (double)ord2f(fenc[lane]) - zk;
        ek = (int)(unsigned)(ekey[lane] & 0xffffffffull);
        if (ek < 0 || ek >= M) { ek = 0; bad = 1; }
        zf_out[lane] = zf;
        I.ideal[lane] = zf;
        I.extreme[lane] = ek;
    }
    int degen = uniform((int)(ballot(bad != 0) != 0));
    if (degen && lane == 0) atomicOr(&ctrl->status, ST_INTERNAL);
    // row i of E in lane i: A[j] = f(e_i)_j - z_j, right-hand side 1
    double A[MO];
    double rhs = 1.0;
#pragma unroll
    for (int j = 0; j < MO; ++j) {
        const double zj = read_lane_f64(zk, j);
        A[j] = lane < MO ? (double)F[(size_t)ek * MO + j] - zj : 0.0;
    }
    // largest |entry| per column of the original matrix
    double colmax[MO];
#pragma unroll
    for (int j = 0; j < MO; ++j) {
        const u64 key = lane < MO ? (u64)__double_as_longlong(fabs(A[j])) : 0ull;
        colmax[j] = __longlong_as_double((long long)wave_max_u64(key));
    }
    // Rows stay in their lanes; pos is the row's position in the eliminated
    // matrix (a swap of two positions exchanges two lanes' pos values).
    int pos = lane;
#pragma unroll
    for (int c = 0; c < MO; ++c) {
        if (degen) break;
        // pivot: largest |A[i][c]| over positions i >= c, least position on ties
        const bool cand = lane < MO && pos >= c;
        const u64 key = cand ? (u64)__double_as_longlong(fabs(A[c])) : 0ull;
        const u64 best = wave_max_u64(key);
        const int piv = (int)wave_min_u32(cand && key == best ? (unsigned)pos : 0xffffffffu);
        const double pv = __longlong_as_double((long long)best);
        if (colmax[c] == 0.0 || pv < 1e-10 * colmax[c]) {
            degen = 1;
            break;
        }
        const int lp = __ffsll((long long)ballot(lane < MO && pos == piv)) - 1;  // pivot row's lane
        const int lc = __ffsll((long long)ballot(lane < MO && pos == c)) - 1;    // position c's lane
        if (piv != c) {
            if (lane == lp) pos = c;
            else if (lane == lc) pos = piv;
        }
        const double acc = read_lane_f64(A[c], lp);
        const double rc = read_lane_f64(rhs, lp);
        const bool below = lane < MO && pos > c;
        const double f = below ? A[c] / acc : 0.0;
#pragma unroll
        for (int j = c; j < MO; ++j) {
            const double acj = read_lane_f64(A[j], lp);
            if (below) A[j] = __dsub_rn(A[j], __dmul_rn(f, acj));
        }
        if (below) rhs = __dsub_rn(rhs, __dmul_rn(f, rc));
    }
    double b[MO];
    if (!degen) {
#pragma unroll
        for (int i = MO - 1; i >= 0; --i) {
            const int li = __ffsll((long long)ballot(lane < MO && pos == i)) - 1;  // row at position i
            double s = read_lane_f64(rhs, li);
#pragma unroll
            for (int j = i + 1; j < MO; ++j) s = __dsub_rn(s, __dmul_rn(read_lane_f64(A[j], li), b[j]));
            b[i] = s / read_lane_f64(A[i], li);
        }
    }
    // intercepts, or the per-objective maximum when degenerate
    double ak = 1.0;
#pragma unroll
    for (int k = 0; k < MO; ++k) {
        if (degen) break;
        const double fk = read_lane_f64(fmxk, k);
        if (!(b[k] > 0.0)) { degen = 1; break; }
        const double a = 1.0 / b[k];
        if (!isfinite(a) || a < 1e-6 * fk) { degen = 1; break; }
        if (k == lane) ak = a;
    }
    if (degen) ak = fmxk > 0.0 ? fmxk : 1.0;
    if (lane < MO) {
        I.intercept[lane] = ak;
        recip_out[lane] = (float)(1.0 / ak);
    }
    if (lane == 0) *I.degenerate = degen;
}

// The squared perpendicular distance of the point f (normalized objectives)
// to the unit direction j (objective k at wn[k * Hp + j]), from the explicit
// residual r = f - (f . w) w. Every caller forms it with this one sequence of
// float32 operations, so a recomputed distance has the same bits.
template <int MO, typename Ptr>
__device__ __forceinline__ float assoc_d2(const float (&f)[MO], Ptr wn, int Hp, int j) {
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
    return d2;
}

// One reference against f; keeps the least distance (strictly less: the
// least j among equal distances when j ascends).
template <int MO, typename Ptr>
__device__ __forceinline__ void assoc_ref(const float (&f)[MO], Ptr wn, int Hp, int j,
                                          float &best, int &bj) {
    const float d2 = assoc_d2<MO>(f, wn, Hp, j);
    if (d2 < best) { best = d2; bj = j; }
}

// (a << 1) | bit(lane) for every lane, with the bits taken from a wave mask:
// one v_addc with the mask as carry-in (a + a + carry).
__device__ __forceinline__ unsigned shift_in(unsigned a, u64 mask) {
    unsigned r;
    u64 carry_out;
    asm("v_addc_co_u32 %0, %1, %2, %2, %3" : "=v"(r), "=s"(carry_out) : "v"(a), "s"(mask));
    return r;
}

// One step of a radix select, run by one full wave: over the 256 counts of
// hist (digits of the keys that match the prefix so far), the digit d at
// which the running count first reaches `need`, and need minus the count of
// the digits below d. Lane t holds bins 4t .. 4t + 3; one wave scan.
__device__ __forceinline__ void hist_digit(const unsigned *hist, int need, int &digit,
                                           int &rest) {
    const int lane = lane_id();
    int h[4], sum = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        h[q] = (int)hist[4 * lane + q];
        sum += h[q];
    }
    const int incl = wave_incl_scan(sum);
    const u64 reach = ballot(incl >= need);
    const int L = reach ? __ffsll((long long)reach) - 1 : 63;
    int acc = __builtin_amdgcn_readlane(incl - sum, L), d = 4 * L + 3;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int hq = __builtin_amdgcn_readlane(h[q], L);
        if (acc + hq >= need) { d = 4 * L + q; break; }
        acc += hq;
    }
    digit = d;
    rest = need - acc;
}

}  // namespace nsga3
