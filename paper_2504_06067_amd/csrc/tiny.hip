// The whole selection of one small instance in one workgroup (Algorithm 1's
// selection of P_{t+1} from R_t: non-dominated sort and front fill,
// normalization, association, niching), for instances whose multi-kernel
// selection would be bound by launch latency rather than by work: at
// 2N = 184 the arithmetic takes a few microseconds on one compute unit,
// while eleven launches take over sixty.
//
// Everything stays in LDS: the objectives, the unit reference directions,
// each point's dominator bits (the full square of 64 x 64 tiles, quarter
// tiles spread over the 16 waves), the fronts, the association keys, the
// niche counts and the candidate segments. The floating-point steps are the multi-kernel path's
// own (the same ASF operations, the intercept solve of norm_solve, the
// residual of assoc_ref), so a small instance gives bit-identical results
// on either path. The niche fill is the same closed form: L* by bisection
// over P(L), the r least tag-1 keys at L* by ranking T's keys in LDS, then
// each reference's picks (nearest at niche count 0, keyed otherwise).
#include <limits.h>

#include "steps.h"

namespace nsga3 {

constexpr int TINY_M = 256;                  // points
constexpr int TINY_W = TINY_M / 64;          // 64-point blocks
constexpr int TINY_H = 2048;                 // references
constexpr int TINY_WN = 8192;                // floats of unit directions (H x m)
constexpr int TINY_THREADS = 1024;
constexpr int TINY_WAVES = TINY_THREADS / 64;
// Work budget of the one-workgroup path in lane operations (about 25 us on
// one compute unit); larger instances fill the chip with the multi-kernel path.
constexpr long long TINY_WORK = 4000000;

// Makes every lane's earlier LDS writes visible to the other lanes of the
// wave before any later read.
__device__ __forceinline__ void tiny_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Position of the k-th (0-based) set bit of w (k below the popcount): halves
// of 32, 16, .. 1 bits, keeping the half that holds it.
__device__ __forceinline__ int tiny_select_bit(u64 w, int k) {
    int pos = 0;
#pragma unroll
    for (int width = 32; width >= 1; width >>= 1) {
        const int c = __popcll(w & ((1ull << width) - 1));
        if (k >= c) {
            k -= c;
            w >>= width;
            pos += width;
        }
    }
    return pos;
}

template <int MO>
__global__ __launch_bounds__(TINY_THREADS) void k_select_tiny(const Inst I) {
    __shared__ float sF[TINY_M * MO];        // objectives [x][k]
    __shared__ __align__(16) float sW[TINY_WN];  // unit directions [k][j] (stride H); later T's keys
    __shared__ u64 sDom[TINY_M * TINY_W];    // point x, word w: bit b = point 64w+b dominates x
    __shared__ u64 sFront[TINY_W];           // members of the current front
    __shared__ u64 sPicked[TINY_W];          // last-front members picked
    __shared__ int sRank[TINY_M];
    __shared__ int sPi[TINY_M];
    __shared__ int sPl[TINY_M];              // reference of a last-front member, else -1
    __shared__ float sD[TINY_M];
    __shared__ u64 sKey[TINY_M];             // association: (d^2 bits << 32) | reference
    __shared__ int sRho[TINY_H], sCnt[TINY_H], sOff[TINY_H], sTp[TINY_H];
    __shared__ int sMemb[TINY_M];            // last-front members by reference, ascending
    __shared__ unsigned sLo[NARROW_M], sHi[NARROW_M];
    __shared__ u64 sExt[NARROW_M];
    __shared__ float sZf[NARROW_M], sRc[NARROW_M];  // ideal point and 1 / a from the solve
    __shared__ int red[TINY_WAVES];
    __shared__ int sVal[4];                  // status bits, size of T, -, scan carry

    const int tid = threadIdx.x, lane = lane_id(), wv = tid >> 6;
    const int M = I.M, H = I.H, N = I.N;
    const int W = (M + 63) >> 6;
    const u64 seed = I.seed;
    Ctrl *ctrl = I.P.ctrl;

    // --- start: status, inputs to LDS (finiteness, reference rows)
    if (tid == 0) {
        ctrl->status = 0;
        sVal[0] = 0;
    }
    if (tid < NARROW_M) {
        sLo[tid] = 0xffffffffu;
        sHi[tid] = 0u;
        sExt[tid] = ~0ull;
    }
    if (tid < TINY_W) sPicked[tid] = 0ull;
    for (int x = tid; x < M; x += TINY_THREADS) sKey[x] = ~0ull;
    for (int j = tid; j < H; j += TINY_THREADS) {
        sRho[j] = 0;
        sCnt[j] = 0;
    }
    int bad = 0;
    for (int e = tid; e < M * MO; e += TINY_THREADS) {
        const float v = I.F[e];
        bad |= isfinite(v) ? 0 : ST_NONFINITE;
        sF[e] = v;
    }
    // column points past M (to the end of their 64-point block) hold +inf
    // and dominate nothing
    for (int e = M * MO + tid; e < W * 64 * MO; e += TINY_THREADS) sF[e] = INFINITY;
    for (int j = tid; j < H; j += TINY_THREADS) {
        // the unit directions of the preparation kernel, operation for operation
        float s = 0.0f;
        bool br = false;
        for (int k = 0; k < MO; ++k) {
            const float v = I.Z[(size_t)j * MO + k];
            br |= !(v >= 0.0f) || !isfinite(v);
            s = fmaf(v, v, s);
        }
        br |= !(s > 0.0f);
        const float inv = br ? 0.0f : 1.0f / sqrtf(s);
        for (int k = 0; k < MO; ++k) sW[k * H + j] = I.Z[(size_t)j * MO + k] * inv;
        if (br) bad |= ST_BADREF;
    }
    lds_barrier();
    if (bad) atomicOr(&sVal[0], bad);
    lds_barrier();
    {
        const int st = uniform(sVal[0]);
        if (st) {
            if (tid == 0) atomicOr(&ctrl->status, st);
            return;
        }
    }

    // --- dominance: task (jb, ib, q) takes row block jb (points in the
    // lanes) against the 16 column points 64 ib + 16 q .. + 15 of block ib,
    // read from LDS at one address per wave (a broadcast); the tasks (the
    // four quarters of every tile of the full square) go round the 16 waves
    for (int task = wv; task < 4 * W * W; task += TINY_WAVES) {
        const int jb = task / (4 * W), ib = (task / 4) % W, q = task & 3;
        const int j = jb * 64 + lane;
        const int c0 = uniform(ib * 64 + 16 * q);
        float fj[MO];
#pragma unroll
        for (int k = 0; k < MO; ++k) fj[k] = j < M ? sF[j * MO + k] : INFINITY;
        // R runs 15 down to 0, so the shifted-in bit of column point c0 + R
        // lands at bit R
        unsigned A = 0;  // bit R: point c0 + R dominates j
#pragma unroll 4
        for (int R = 15; R >= 0; --R) {
            u64 lt = 0, gt = 0;
#pragma unroll
            for (int k = 0; k < MO; ++k) {
                const float x = sF[(c0 + R) * MO + k];
                lt |= ballot(x < fj[k]);
                gt |= ballot(x > fj[k]);
            }
            A = shift_in(A, lt & ~gt);
        }
        if (j < M) ((unsigned short *)sDom)[(j * TINY_W + ib) * 4 + q] = (unsigned short)A;
    }
    lds_barrier();
    // --- fronts: point x = tid (waves 0 .. W-1); front k = alive points
    // without an alive dominator; stop at the first l with |F_0..F_l| >= N
    const bool own = tid < M;
    int cnt = 0;
    bool alive = own;
    if (own)
        for (int w = 0; w < W; ++w) cnt += __popcll(sDom[tid * TINY_W + w]);
    int myrank = NSGA3_UNRANKED;
    int l = 0, S = 0, cum = 0;
    for (int k = 0;; ++k) {
        const bool newly = alive && cnt == 0;
        const u64 bal = ballot(newly);
        if (wv < W && lane == 0) sFront[wv] = bal;
        lds_barrier();
        int size = 0;
        for (int w = 0; w < W; ++w) size += __popcll(uniform(sFront[w]));
        if (newly) {
            myrank = k;
            alive = false;
        }
        if (size == 0 || cum + size >= N) {
            if (size == 0 && tid == 0) atomicOr(&ctrl->status, ST_INTERNAL);
            l = k;
            S = cum;
            break;
        }
        cum += size;
        if (alive)
            for (int w = 0; w < W; ++w) cnt -= __popcll(sDom[tid * TINY_W + w] & sFront[w]);
        lds_barrier();  // sFront is rewritten
    }
    if (own) sRank[tid] = myrank;
    const bool in_st = own && myrank <= l;

    // --- normalization over S_t: ideal point and maxima, ASF extreme points
    // (the float operations of the multi-kernel path), the FP64 solve
#pragma unroll
    for (int k = 0; k < MO; ++k) {
        const float v = in_st ? sF[tid * MO + k] : 0.0f;
        const unsigned lo = wave_min_u32(in_st ? f2ord(v) : 0xffffffffu);
        const unsigned hi = wave_max_u32(in_st ? f2ord(v) : 0u);
        if (lane == 0 && wv < W) {
            atomicMin(&sLo[k], lo);
            atomicMax(&sHi[k], hi);
        }
    }
    lds_barrier();
    {
        float fp[MO], g[MO];
#pragma unroll
        for (int k = 0; k < MO; ++k) {
            const float v = in_st ? sF[tid * MO + k] : 0.0f;
            fp[k] = in_st ? v - ord2f(sLo[k]) : 0.0f;
            g[k] = 1e6f * fp[k];
        }
        float g1 = g[0], g2 = -INFINITY;
        int p1 = 0;
#pragma unroll
        for (int k = 1; k < MO; ++k) {
            if (g[k] > g1) { g2 = g1; g1 = g[k]; p1 = k; }
            else if (g[k] > g2) g2 = g[k];
        }
#pragma unroll
        for (int k = 0; k < MO; ++k) {
            const float asf = fmaxf(fp[k], k == p1 ? g2 : g1);
            const u64 key = in_st ? (((u64)__float_as_uint(asf) << 32) | (unsigned)tid) : ~0ull;
            const u64 wkey = wave_min_u64(key);
            if (lane == 0 && wv < W) atomicMin(&sExt[k], wkey);
        }
    }
    lds_barrier();
    if (wv == 0) norm_solve<MO>(I, sLo, sHi, sExt, sF, sZf, sRc);
    lds_barrier();  // zf and recip are written by wave 0

    // --- association: point slot tid % TINY_M, reference quarter tid / TINY_M
    {
        const int x = tid % TINY_M, q = tid / TINY_M;
        if (x < M && sRank[x] <= l) {
            float f[MO];
#pragma unroll
            for (int k = 0; k < MO; ++k) f[k] = (sF[x * MO + k] - sZf[k]) * sRc[k];
            const int R = (H + 3) / 4;
            const int h0 = q * R, h1 = min(H, h0 + R);
            float best = INFINITY;
            int bj = h0;
            int j = h0;
            for (; j + 4 <= h1; j += 4) {
                assoc_ref<MO>(f, (const float *)sW, H, j, best, bj);
                assoc_ref<MO>(f, (const float *)sW, H, j + 1, best, bj);
                assoc_ref<MO>(f, (const float *)sW, H, j + 2, best, bj);
                assoc_ref<MO>(f, (const float *)sW, H, j + 3, best, bj);
            }
            for (; j < h1; ++j) assoc_ref<MO>(f, (const float *)sW, H, j, best, bj);
            if (h0 < h1) atomicMin(&sKey[x], ((u64)__float_as_uint(best) << 32) | (unsigned)bj);
        }
    }
    lds_barrier();
    bad = 0;
    if (own) {
        int pj = -1;
        float d = -1.0f;
        if (in_st) {
            const u64 key = sKey[tid];
            pj = (int)(unsigned)(key & 0xffffffffull);
            if (pj < 0 || pj >= H) {
                bad = ST_INTERNAL;
                pj = 0;
            }
            d = sqrtf(__uint_as_float((unsigned)(key >> 32)));
            atomicAdd(myrank < l ? &sRho[pj] : &sCnt[pj], 1);
        }
        sPi[tid] = pj;
        sPl[tid] = myrank == l ? pj : -1;
        sD[tid] = d;
        I.pi[tid] = pj;
        I.dist[tid] = d;
        I.rank[tid] = myrank;
    }
    lds_barrier();

    // --- niche fill, planned by wave 0 alone (wave reductions, no block
    // barriers): lane L owns the references [L*S, (L+1)*S); CSR offsets in
    // reference order, L* = max{L : P(L) <= K} by bisection, the r least
    // tag-1 keys of T at L*, and the picks t_j of every reference (sTp)
    const int K = N - S;
    if (wv == 0) {
        const int SP = (H + 63) / 64;
        const int j0 = min(H, lane * SP), j1 = min(H, j0 + SP);
        int csum = 0, cmax = 0;
        for (int j = j0; j < j1; ++j) {
            const int c = sCnt[j];
            csum += c;
            if (c > 0) cmax = max(cmax, sRho[j] + c);
        }
        const int incl = wave_incl_scan(csum);
        int run = incl - csum;
        for (int j = j0; j < j1; ++j) {
            sOff[j] = run;
            run += sCnt[j];
        }
        const int total = uniform(__builtin_amdgcn_readlane(incl, 63));
        if (K >= total) {
            for (int j = j0; j < j1; ++j) sTp[j] = sCnt[j];
            if (lane == 0 && K > total) atomicOr(&ctrl->status, ST_INTERNAL);
        } else {
            // P(lo) <= K < P(hi)
            int lo = 0, hi = (int)wave_max_u32((unsigned)cmax);
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                int p = 0;
                for (int j = j0; j < j1; ++j) p += min(sCnt[j], max(0, mid - sRho[j]));
                if (uniform(wave_sum(p)) <= K) lo = mid;
                else hi = mid;
            }
            const int Ls = lo;
            int pl = 0, tcount = 0;
            for (int j = j0; j < j1; ++j) {
                const int c = sCnt[j], rh = sRho[j];
                const int t = min(c, max(0, Ls - rh));
                pl += t;
                tcount += (c > 0 && rh <= Ls && Ls < rh + c);
                sTp[j] = t;
            }
            pl = uniform(wave_sum(pl));
            const int tsize = uniform(wave_sum(tcount));
            const int r = K - pl;
            // T's keys gathered in LDS (the unit directions' space is free
            // now: keys at [0, 16 KB), references at [16 KB, 24 KB)); a key
            // of T is among the r least when fewer than r keys are smaller
            // (keys of distinct references differ)
            u64 *tkey = (u64 *)sW;
            int *tref = (int *)(sW + 2 * TINY_H);
            if (r > 0 && r >= tsize) {
                for (int j = j0; j < j1; ++j) {
                    const int c = sCnt[j], rh = sRho[j];
                    if (c > 0 && rh <= Ls && Ls < rh + c) sTp[j] += 1;
                }
            } else if (r > 0) {
                if (lane == 0) sVal[1] = 0;
                tiny_wave_sync();
                for (int j = j0; j < j1; ++j) {
                    const int c = sCnt[j], rh = sRho[j];
                    if (!(c > 0 && rh <= Ls && Ls < rh + c)) continue;
                    const int e = atomicAdd(&sVal[1], 1);
                    tkey[e] = tie_key(seed, 1u, (unsigned)j, (unsigned)Ls);
                    tref[e] = j;
                }
                tiny_wave_sync();
                for (int e = lane; e < tsize; e += 64) {
                    const u64 mine = tkey[e];
                    int rank = 0;
#pragma unroll 8
                    for (int v = 0; v < tsize; ++v) rank += tkey[v] < mine;
                    if (rank < r) sTp[tref[e]] += 1;
                }
            }
        }
    }
    lds_barrier();  // offsets and picks per reference are complete
    // the rank among the remaining candidates of every keyed pick, computed
    // up front in parallel (the association keys are no longer needed):
    // pick i of reference j, at level rho_j + i, is stored at sOff[j] + i;
    // each member's distance is copied to its segment slot
    int *sPickRank = (int *)sKey;
    float *sSegD = (float *)sKey + TINY_M;
    if (own && myrank == l) {
        // slot: last-front members of the same reference with a smaller index
        const int p = sPi[tid];
        int slot = 0;
#pragma unroll 8
        for (int y = 0; y < tid; ++y) slot += sPl[y] == p;
        sMemb[sOff[p] + slot] = tid;
        sSegD[sOff[p] + slot] = sD[tid];
        const int rh = sRho[p];
        if (slot < sTp[p] && rh + slot > 0)
            sPickRank[sOff[p] + slot] =
                (int)(tie_key(seed, 2u, (unsigned)p, (unsigned)(rh + slot)) %
                      (u64)(sCnt[p] - slot));
    }
    lds_barrier();  // the segments and pick ranks are complete
    for (int j = tid; j < H; j += TINY_THREADS) {
        const int t = sTp[j], c = sCnt[j], rh = sRho[j];
        if (t <= 0) continue;
        const int *seg = sMemb + sOff[j];
        if (t >= c) {
            for (int i = 0; i < c; ++i) atomicOr(&sPicked[seg[i] >> 6], 1ull << (seg[i] & 63));
            continue;
        }
        u64 rem[TINY_W];
#pragma unroll
        for (int w = 0; w < TINY_W; ++w) {
            const int v = c - 64 * w;
            rem[w] = v >= 64 ? ~0ull : (v > 0 ? ((1ull << v) - 1) : 0ull);
        }
        for (int lev = rh; lev < rh + t; ++lev) {
            int pos = -1;
            if (lev == 0) {
                // the nearest candidate (least distance, then least index)
                u64 best = ~0ull;
                const float *segd = sSegD + sOff[j];
                for (int i = 0; i < c; ++i) {
                    const u64 k = ((u64)__float_as_uint(segd[i]) << 32) | (unsigned)i;
                    best = k < best ? k : best;
                }
                pos = (int)(unsigned)(best & 0xffffffffull);
            } else {
                int kk = sPickRank[sOff[j] + (lev - rh)];
#pragma unroll
                for (int w = 0; w < TINY_W; ++w) {
                    const int pc = __popcll(rem[w]);
                    if (pos < 0 && kk < pc) pos = 64 * w + tiny_select_bit(rem[w], kk);
                    else if (pos < 0) kk -= pc;
                }
            }
            if (pos < 0 || pos >= c) {
                atomicOr(&ctrl->status, ST_INTERNAL);
                break;
            }
#pragma unroll
            for (int w = 0; w < TINY_W; ++w)
                if (w == (pos >> 6)) rem[w] &= ~(1ull << (pos & 63));
            const int x = seg[pos];
            atomicOr(&sPicked[x >> 6], 1ull << (x & 63));
        }
    }
    lds_barrier();

    // --- output: S and the picks, ascending
    {
        const bool sel = own && (myrank < l || ((sPicked[tid >> 6] >> (tid & 63)) & 1ull));
        const u64 bal = ballot(sel);
        if (wv < W && lane == 0) red[wv] = __popcll(bal);
        lds_barrier();
        int pos = 0, tot = 0;
        for (int v = 0; v < W; ++v) {
            const int c = (int)red[v];
            if (v < wv) pos += c;
            tot += c;
        }
        pos += mbcnt(bal);
        if (sel && pos < N) I.selected[pos] = tid;
        if (tid == 0) {
            I.front_info[0] = l;
            I.front_info[1] = S;
            I.front_info[2] = N - S;
            I.front_info[3] = l + 1;
            if (tot != N) atomicOr(&ctrl->status, ST_INTERNAL);
        }
        if (bad) atomicOr(&ctrl->status, bad);
    }
}

bool tiny_fits(int M, int m, int H) {
    if (M > TINY_M || m > NARROW_M || H > TINY_H || (long long)H * m > TINY_WN) return false;
    // one compute unit's work: dominance (2m + 1 per pair of the square) and
    // association (about 3m + 3 per point and reference)
    const long long work = (long long)M * M * (2 * m + 1) + (long long)M * H * (3 * m + 3);
    return work <= TINY_WORK;
}

hipError_t launch_select_tiny(const Inst &I, hipStream_t s) {
    switch (I.m) {
#define NSGA3_TINY_CASE(MO)                                                                   \
    case MO:                                                                                  \
        NSGA3_LAUNCH("select_tiny", k_select_tiny<MO>, dim3(1), dim3(TINY_THREADS), 0, s, I); \
        break;
        NSGA3_TINY_CASE(2) NSGA3_TINY_CASE(3) NSGA3_TINY_CASE(4) NSGA3_TINY_CASE(5)
        NSGA3_TINY_CASE(6) NSGA3_TINY_CASE(7) NSGA3_TINY_CASE(8) NSGA3_TINY_CASE(9)
        NSGA3_TINY_CASE(10) NSGA3_TINY_CASE(11) NSGA3_TINY_CASE(12) NSGA3_TINY_CASE(13)
        NSGA3_TINY_CASE(14) NSGA3_TINY_CASE(15) NSGA3_TINY_CASE(16)
#undef NSGA3_TINY_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace nsga3
