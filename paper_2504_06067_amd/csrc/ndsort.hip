// Non-dominated sorting (paper Sec. II-C; Algorithm 1 "Non-dominated-sort")
// as a bit-packed dominance matrix followed by front peeling, for a batch of
// independent instances.
//
// The points are first placed in ascending buckets of their first objective
// (see "point placement" below); the matrix and the peel work on positions.
// Dominance matrix layout ("word-major"): mask[w * Mp + j] is a 64-bit word
// whose bit b is set iff position 64*w + b dominates position j. A wave of 64
// consecutive j therefore reads or writes 512 contiguous bytes.
//
// Kernels:
//   k_init           per instance: control block, peel counters, front_info,
//                    placement counts
//   k_prep           points: finiteness, +inf padding of the objective copy,
//                    dominator counts, ranks, the peel's front ring, niche
//                    flags, placement bucket counts; references: unit
//                    directions and their check, niche counters
//   k_place_scatter  each point's position; the objective copy (small copies),
//                    the position-to-point map, per-block tile bounds
//   k_place_gather   the objective copy in position order (large copies)
//   k_dominance      triangle of 64x64 tiles: ordered tiles (one direction,
//                    m - 1 compares per pair, ANDed in EXEC by a v_cmpx
//                    chain from m = 5), the rest with both directions from
//                    one set of 2m compares (two v_cmpx chains from m = 5);
//                    fused dominator counts
//   k_dominance_wide the same for m > NARROW_M, objectives in chunks
//   k_peel           fronts of every instance, persistent over its chunks
#include <mutex>
#include <utility>

#include "steps.h"

namespace nsga3 {

long long dominance_tiles(int W) { return (long long)W * (W + 1) / 2; }

__global__ __launch_bounds__(256) void k_init(BatchView bv) {
    CInst &I = bv.tab[blockIdx.x];
    init_instance(I.P.ctrl, I.front_info, I.n_stop, bv.run, I.P.bcount, threadIdx.x);
    static_assert(TICKET_SHARDS * PEEL_PIPE_GROUPS <= 256, "one word per thread");
    if (blockIdx.x == 0 && threadIdx.x < TICKET_SHARDS * PEEL_PIPE_GROUPS)
        bv.ticket[(threadIdx.x % TICKET_SHARDS) * TICKET_STRIDE + threadIdx.x / TICKET_SHARDS] = 0;
}

// ------------------------------------------------------- point placement
//
// The dominance and the peel work on positions, not on point indices: the
// points are placed in ascending buckets of their first objective,
//   bucket(x) = floor((f_1(x) - lo) * PLACE_BUCKETS / (hi - lo)), clamped,
// (lo, hi: least and largest f_1 of a strided sample of 256 points), a
// monotone function of f_1 in float32. k_prep counts the buckets, and
// k_place_scatter places the points (k_place_gather writes large objective
// copies in position order).
// A point in a lower bucket has a strictly smaller f_1, so it cannot be
// dominated by a point of a higher bucket. For a tile whose column block
// lies wholly in lower buckets than its row block ("ordered") one direction
// of the relation is known to be empty and the other needs no compare of f_1.
// Within a bucket the positions follow the order of arrival; ranks do not
// depend on positions, only the internal matrix does.

// Largest objective copy written by scattered stores (one L2 of an XCD).
constexpr long long PLACE_SCATTER_BYTES = 4ll << 20;

__device__ __forceinline__ int place_bucket(float x, float lo, float scale) {
    const float t = (x - lo) * scale;
    return t >= (float)PLACE_BUCKETS ? PLACE_BUCKETS - 1 : (t > 0.0f ? (int)t : 0);
}

// Grid: [all instances' padded points][all instances' padded references].
__global__ __launch_bounds__(256) void k_prep(BatchView bv, int npt) {
    const bool points = (int)(blockIdx.x * blockDim.x) < npt;
    if (points) {
        const Local L = locate(bv.pt_pref, bv.B);
        CInst &I = bv.tab[L.b];
        const int j = L.i, M = I.M, m = I.m, Mp = I.Mp;
        bool bad = false;
        // In a whole selection the ideal point is the least value of each
        // objective over all points: a point that attains the least value
        // and is not dominated among those that attain it is not dominated
        // at all, so it is in front 0 and the least value over S_t is the
        // same float. Reduced per wave, then per block in LDS: one atomic
        // per block and objective (atomics on one address serialize).
        const bool ideal_here = (bv.run & RUN_ND) && (bv.run & RUN_NORM) && m <= NARROW_M;
        __shared__ unsigned s_lo[4][NARROW_M];
        __shared__ unsigned s_rng[2][4];
        __shared__ unsigned hist[PLACE_BUCKETS];
        const int wv = threadIdx.x >> 6;
        if (ideal_here && lane_id() < m) s_lo[wv][lane_id()] = 0xffffffffu;
        float f1 = 0.0f;  // this point's first objective
        if (j < Mp && (bv.run & RUN_ND)) {
            for (int k = 0; k < m; ++k) {
                float v = INFINITY;
                if (j < M) {
                    v = I.F[(size_t)j * m + k];
                    bad |= !isfinite(v);
                } else {
                    // padding positions (the placement fills positions < M)
                    I.P.ft[((size_t)(j >> 6) * m + k) * 64 + (j & 63)] = v;
                }
                if (k == 0) f1 = v;
                if (ideal_here) {
                    const unsigned lo = wave_min_u32(j < M ? f2ord(v) : 0xffffffffu);
                    if (lane_id() == 0) s_lo[wv][k] = lo;
                }
            }
            I.P.nd[j] = 0;
            if (j < M) I.rank[j] = NSGA3_UNRANKED;
            if ((j & 63) == 0) {
                // no word of the front ring may carry a tag of this call yet
                u64 *ring = I.P.ring + (size_t)(j >> 5);
                const size_t sw = (size_t)front_slot_words(I.W);
#pragma unroll
                for (int r = 0; r < PEEL_RING; ++r) {
                    ring[r * sw] = 0ull;
                    ring[r * sw + 1] = 0ull;
                }
            }
        }
        if (bv.run & RUN_ND) {
            // (the run flags and the points branch are uniform over the block)
            // Placement counts (see k_place_scatter). The bucket range is that
            // of a strided sample of 256 points, the same in every block, so
            // no pass over all points precedes the bucketing; points outside
            // it clamp to the end buckets, which keeps the bucket function
            // monotone (the range only decides how many tiles are ordered).
            const int js = (int)(((long long)threadIdx.x * M) >> 8);
            const unsigned sv = f2ord(I.F[(size_t)js * m]);
            const unsigned wlo = wave_min_u32(sv), whi = wave_max_u32(sv);
            if (lane_id() == 0) {
                s_rng[0][wv] = wlo;
                s_rng[1][wv] = whi;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) hist[threadIdx.x + 256 * q] = 0;
            lds_barrier();
            if (ideal_here && (int)threadIdx.x < m) {
                const int k = threadIdx.x;
                const unsigned lo = min(min(s_lo[0][k], s_lo[1][k]), min(s_lo[2][k], s_lo[3][k]));
                if (lo != 0xffffffffu) atomicMin(&I.P.ctrl->zmin_enc[k], lo);
            }
            const float lo = ord2f(min(min(s_rng[0][0], s_rng[0][1]), min(s_rng[0][2], s_rng[0][3])));
            const float hi = ord2f(max(max(s_rng[1][0], s_rng[1][1]), max(s_rng[1][2], s_rng[1][3])));
            const float span = hi - lo;
            const float scale = span > 0.0f && span < INFINITY ? (float)PLACE_BUCKETS / span : 0.0f;
            int b = 0;
            unsigned r = 0;
            if (j < M) {
                b = place_bucket(f1, lo, scale);
                r = atomicAdd(&hist[b], 1u);  // rank within the bucket and block
            }
            lds_barrier();
            // the thread's four bins: one global atomic per nonempty bin
            // reserves the block's run of the bucket (all four in flight)
            unsigned cq[4], base[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) cq[q] = hist[threadIdx.x + 256 * q];
#pragma unroll
            for (int q = 0; q < 4; ++q)
                base[q] = cq[q] ? atomicAdd(&I.P.bcount[threadIdx.x + 256 * q], cq[q]) : 0u;
#pragma unroll
            for (int q = 0; q < 4; ++q) hist[threadIdx.x + 256 * q] = base[q];
            lds_barrier();
            if (j < M) I.P.pkey[j] = ((unsigned)b << PLACE_RANK_BITS) | (hist[b] + r);
        }
        if (j < M && (bv.run & RUN_NICHE)) {
            I.P.picked[j] = 0;
            if (j % COMPACT_TILE == 0) I.P.tcnt[j / COMPACT_TILE] = 0;
        }
        if (ballot(bad) != 0 && lane_id() == 0) atomicOr(&I.P.ctrl->status, ST_NONFINITE);
    } else {
        const int base = uniform((int)(blockIdx.x * blockDim.x)) - npt;
        const int b = uniform(find_range(bv.ref_pref, bv.B, base));
        CInst &I = bv.tab[b];
        const int t = base - bv.ref_pref[b] + (int)threadIdx.x;
        const int H = I.H, Hp = I.Hp, m = I.m;
        bool bad = false;
        if (t < Hp && (bv.run & RUN_ASSOC)) {
            // unit reference directions; padding repeats the last real one
            const int j = t < H ? t : H - 1;
            float s = 0.0f;
            for (int k = 0; k < m; ++k) {
                const float v = I.Z[(size_t)j * m + k];
                bad |= !(v >= 0.0f) || !isfinite(v);
                s = fmaf(v, v, s);
            }
            bad |= !(s > 0.0f);
            const float inv = bad ? 0.0f : 1.0f / sqrtf(s);
            // structure of arrays for the specialized association kernels (a
            // wave reads one objective of consecutive references), rows for
            // the general one (a wave reads consecutive objectives of one)
            for (int k = 0; k < m; ++k) {
                const size_t at = m <= NARROW_M ? (size_t)k * Hp + t : (size_t)t * m + k;
                I.P.wn[at] = I.Z[(size_t)j * m + k] * inv;
            }
        }
        if (t < H && (bv.run & RUN_NICHE)) {
            I.P.rho[t] = 0;
            I.P.cnt[t] = 0;
            I.P.fill[t] = 0;
        }
        if (ballot(bad) != 0 && lane_id() == 0) atomicOr(&I.P.ctrl->status, ST_BADREF);
    }
}

// Every block scans the instance's bucket counts into bucket starts, then
// each point goes to its position: the objective copy (blocks of 64
// positions, objective-major within a block), the position's point, and the
// tile bounds of the position's block (from its first and its last point).
// copy: the point also writes its objectives at the position (a scattered
// 4-byte store per objective); otherwise k_place_gather writes the copy.
__global__ __launch_bounds__(256) void k_place_scatter(BatchView bv, int copy) {
    __shared__ int start[PLACE_BUCKETS + 1];
    __shared__ int wsum[4];
    const Local L = locate(bv.pt_pref, bv.B);
    CInst &I = bv.tab[L.b];
    const int j = L.i, M = I.M, m = I.m;
    const int t = threadIdx.x, wv = t >> 6;
    int c[4], sum = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        c[q] = (int)I.P.bcount[4 * t + q];
        sum += c[q];
    }
    const int incl = wave_incl_scan(sum);
    if (lane_id() == 63) wsum[wv] = incl;
    lds_barrier();
    int run = incl - sum;
    for (int v = 0; v < wv; ++v) run += wsum[v];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        start[4 * t + q] = run;
        run += c[q];
    }
    if (t == 255) start[PLACE_BUCKETS] = run;
    lds_barrier();
    if (j < M) {
        const unsigned key = I.P.pkey[j];
        const int b = (int)(key >> PLACE_RANK_BITS);
        const int pos = start[b] + (int)(key & ((1u << PLACE_RANK_BITS) - 1u));
        I.P.perm[pos] = j;
        if (copy) {
            float *dst = I.P.ft + (size_t)(pos >> 6) * m * 64 + (pos & 63);
            for (int k = 0; k < m; ++k) dst[k * 64] = I.F[(size_t)j * m + k];
        }
        // tiles (ib, jb) with every point of ib in a lower bucket than the
        // first point of jb: ib below the block of that bucket's start
        if ((pos & 63) == 0) I.P.row_ord[pos >> 6] = start[b] >> 6;
        // words of column block c from row blocks that start after the
        // bucket of c's last point are zero
        if ((pos & 63) == 63 || pos == M - 1) I.P.col_end[pos >> 6] = (start[b + 1] + 63) >> 6;
    }
}

// The objective copy in position order: each position reads its point's
// row of F (a gather) and the 64 positions of a block write each objective's
// 256 bytes together. For copies larger than the L2, where scattered 4-byte
// stores cost a partial-line write each. Grid: all instances' padded points
// (as positions).
__global__ __launch_bounds__(256) void k_place_gather(BatchView bv) {
    const Local L = locate(bv.pt_pref, bv.B);
    CInst &I = bv.tab[L.b];
    const int pos = L.i, M = I.M, m = I.m;
    if (pos >= M) return;
    const int j = I.P.perm[pos];
    float *dst = I.P.ft + (size_t)(pos >> 6) * m * 64 + (pos & 63);
    const float *src = I.F + (size_t)j * m;
    for (int k = 0; k < m; ++k) dst[k * 64] = src[k];
}

// Lane R of `old` takes the wave-uniform value v.
template <int R>
__device__ __forceinline__ unsigned write_lane(unsigned old, unsigned v) {
    asm("v_writelane_b32 %0, %1, %2" : "+v"(old) : "s"(v), "i"(R));
    return old;
}

// Tiles of the triangle in rows 0 .. jb - 1 (row jb holds tiles ib = 0 .. jb).
__device__ __forceinline__ long long tri(long long jb) { return jb * (jb + 1) / 2; }

// Row of triangle tile t: the largest jb with tri(jb) <= t.
__device__ __forceinline__ int row_of(long long t) {
    long long jb = (long long)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (tri(jb + 1) <= t) ++jb;
    while (tri(jb) > t) --jb;
    return (int)jb;
}

// GW consecutive column values of one objective (one scalar load). The
// group width keeps GW * m values within the scalar register budget (no
// spills, 8 waves per SIMD): the wider the group, the fewer scalar loads per
// column point, which matter most for large m.
template <int MO>
constexpr int col_group() { return MO <= 6 ? 8 : (MO <= 13 ? 4 : 2); }

template <int GW>
struct alignas(4 * GW) ColV {
    float a[GW];
};

// The wave mask of lanes with s_k <= v_k for every k < N (N <= 15), formed
// in EXEC by a chain of v_cmpx (each compare runs only on the lanes that
// passed the ones before it), then EXEC is set back to `saved`, the mask the
// wave entered with. From N = 6 on, a wave with no lane left after four
// compares skips the rest (the mask is then empty either way). One asm
// block, so no other vector instruction runs under the narrowed EXEC;
// unused operand slots repeat slot 0.
template <int N>
__device__ __forceinline__ u64 and_le_exec(const float (&s)[15], const float (&v)[15], u64 saved) {
    static_assert(N >= 1 && N <= 15, "1 to 15 compares");
    u64 res;
#define NSGA3_CMPX(i) ".if " #i " < %c[n]\n v_cmpx_le_f32_e32 vcc, %[s" #i "], %[v" #i "]\n.endif\n"
    asm volatile(NSGA3_CMPX(0) NSGA3_CMPX(1) NSGA3_CMPX(2) NSGA3_CMPX(3)
                 ".if 5 < %c[n]\n s_cbranch_execz 1f\n.endif\n"
                 NSGA3_CMPX(4) NSGA3_CMPX(5) NSGA3_CMPX(6)
                 NSGA3_CMPX(7) NSGA3_CMPX(8) NSGA3_CMPX(9)
                 NSGA3_CMPX(10) NSGA3_CMPX(11) NSGA3_CMPX(12) NSGA3_CMPX(13) NSGA3_CMPX(14)
                 "1:\n"
                 "s_mov_b64 %[res], exec\n"
                 "s_mov_b64 exec, %[save]\n"
                 : [res] "=s"(res)
                 : [n] "i"(N), [save] "s"(saved),
                   [s0] "s"(s[0]), [v0] "v"(v[0]), [s1] "s"(s[1]), [v1] "v"(v[1]),
                   [s2] "s"(s[2]), [v2] "v"(v[2]), [s3] "s"(s[3]), [v3] "v"(v[3]),
                   [s4] "s"(s[4]), [v4] "v"(v[4]), [s5] "s"(s[5]), [v5] "v"(v[5]),
                   [s6] "s"(s[6]), [v6] "v"(v[6]), [s7] "s"(s[7]), [v7] "v"(v[7]),
                   [s8] "s"(s[8]), [v8] "v"(v[8]), [s9] "s"(s[9]), [v9] "v"(v[9]),
                   [s10] "s"(s[10]), [v10] "v"(v[10]), [s11] "s"(s[11]), [v11] "v"(v[11]),
                   [s12] "s"(s[12]), [v12] "v"(v[12]), [s13] "s"(s[13]), [v13] "v"(v[13]),
                   [s14] "s"(s[14]), [v14] "v"(v[14])
                 : "vcc");
#undef NSGA3_CMPX
    return res;
}

// As and_le_exec, with s_k >= v_k.
template <int N>
__device__ __forceinline__ u64 and_ge_exec(const float (&s)[15], const float (&v)[15], u64 saved) {
    static_assert(N >= 1 && N <= 15, "1 to 15 compares");
    u64 res;
#define NSGA3_CMPXG(i) ".if " #i " < %c[n]\n v_cmpx_ge_f32_e32 vcc, %[s" #i "], %[v" #i "]\n.endif\n"
    asm volatile(NSGA3_CMPXG(0) NSGA3_CMPXG(1) NSGA3_CMPXG(2) NSGA3_CMPXG(3)
                 ".if 5 < %c[n]\n s_cbranch_execz 1f\n.endif\n"
                 NSGA3_CMPXG(4) NSGA3_CMPXG(5) NSGA3_CMPXG(6)
                 NSGA3_CMPXG(7) NSGA3_CMPXG(8) NSGA3_CMPXG(9)
                 NSGA3_CMPXG(10) NSGA3_CMPXG(11) NSGA3_CMPXG(12) NSGA3_CMPXG(13) NSGA3_CMPXG(14)
                 "1:\n"
                 "s_mov_b64 %[res], exec\n"
                 "s_mov_b64 exec, %[save]\n"
                 : [res] "=s"(res)
                 : [n] "i"(N), [save] "s"(saved),
                   [s0] "s"(s[0]), [v0] "v"(v[0]), [s1] "s"(s[1]), [v1] "v"(v[1]),
                   [s2] "s"(s[2]), [v2] "v"(v[2]), [s3] "s"(s[3]), [v3] "v"(v[3]),
                   [s4] "s"(s[4]), [v4] "v"(v[4]), [s5] "s"(s[5]), [v5] "v"(v[5]),
                   [s6] "s"(s[6]), [v6] "v"(v[6]), [s7] "s"(s[7]), [v7] "v"(v[7]),
                   [s8] "s"(s[8]), [v8] "v"(v[8]), [s9] "s"(s[9]), [v9] "v"(v[9]),
                   [s10] "s"(s[10]), [v10] "v"(v[10]), [s11] "s"(s[11]), [v11] "v"(v[11]),
                   [s12] "s"(s[12]), [v12] "v"(v[12]), [s13] "s"(s[13]), [v13] "v"(v[13]),
                   [s14] "s"(s[14]), [v14] "v"(v[14])
                 : "vcc");
#undef NSGA3_CMPXG
    return res;
}

// From this many objectives the ordered step ANDs its compares in EXEC:
// m - 1 v_cmpx and two scalar moves per column point, against m - 1 v_cmp
// and m - 2 s_and (the scalar unit issues at the vector unit's rate, so the
// s_and chain competes with the compares at large m).
constexpr int CMPX_MIN_M = 5;

// One compare step against column point i = 64 * ib + R (uniform, objective
// values v[k].a[R % GW]): the wave masks lt = {j : f_i < f_j in some
// objective}, gt = {j : f_i > f_j in some objective} come from 2m compares;
// then
//   i dominates j  <=>  j in lt \ gt   (bit R of lane j's word A)
//   j dominates i  <=>  j in gt \ lt   (the whole mask is row i's word B)
// From CMPX_MIN_M objectives the compares form two EXEC chains instead, le =
// {j : f_i <= f_j in every objective} and ge = {j : f_i >= f_j in every
// objective}, with lt \ gt = le \ ge and gt \ lt = ge \ le.
template <int MO, int GW, int R>
__device__ __forceinline__ void dom_step(const ColV<GW> (&v)[MO], const float (&fj)[MO],
                                         unsigned &a_lo, unsigned &a_hi, unsigned &b_lo,
                                         unsigned &b_hi) {
    u64 i_dom_j, j_dom_i;
    if constexpr (MO >= CMPX_MIN_M && MO <= 16) {
        // all <= (le) and all >= (ge) by EXEC chains: i dominates j when le
        // and not ge (some objective strictly less), j dominates i when ge
        // and not le
        float s[15], w[15];
        const u64 e0 = __builtin_amdgcn_read_exec();
        u64 le = ~0ull, ge = ~0ull;
        {
#pragma unroll
            for (int k = 0; k < 15; ++k) {
                s[k] = k < MO ? v[k].a[R % GW] : v[0].a[R % GW];
                w[k] = k < MO ? fj[k] : fj[0];
            }
        }
        if constexpr (MO <= 15) {
            le = and_le_exec<MO>(s, w, e0);
            ge = and_ge_exec<MO>(s, w, e0);
        } else {
            // the 16th objective by a plain compare
            le = and_le_exec<15>(s, w, e0) & ballot(v[15].a[R % GW] <= fj[15]);
            ge = and_ge_exec<15>(s, w, e0) & ballot(v[15].a[R % GW] >= fj[15]);
        }
        i_dom_j = le & ~ge;
        j_dom_i = ge & ~le;
    } else {
        u64 lt = 0, gt = 0;
#pragma unroll
        for (int k = 0; k < MO; ++k) {
            const float x = v[k].a[R % GW];
            lt |= ballot(x < fj[k]);
            gt |= ballot(x > fj[k]);
        }
        i_dom_j = lt & ~gt;
        j_dom_i = gt & ~lt;
    }
    if (R >= 32) a_hi = shift_in(a_hi, i_dom_j);
    else a_lo = shift_in(a_lo, i_dom_j);
    b_lo = write_lane<R>(b_lo, (unsigned)j_dom_i);
    b_hi = write_lane<R>(b_hi, (unsigned)(j_dom_i >> 32));
}

// Column points GW*g + GW - 1 down to GW*g: their values arrive with one
// scalar load per objective.
template <int MO, int GW, int g, int... Is>
__device__ __forceinline__ void dom_group(std::integer_sequence<int, Is...>,
                                          const NSGA3_RO float *fi, const float (&fj)[MO],
                                          unsigned &a_lo, unsigned &a_hi, unsigned &b_lo,
                                          unsigned &b_hi) {
    ColV<GW> v[MO];
#pragma unroll
    for (int k = 0; k < MO; ++k) {
        const NSGA3_RO ColV<GW> &src = *(const NSGA3_RO ColV<GW> *)(fi + k * 64 + GW * g);
#pragma unroll
        for (int q = 0; q < GW; ++q) v[k].a[q] = src.a[q];
    }
    (dom_step<MO, GW, GW * g + GW - 1 - Is>(v, fj, a_lo, a_hi, b_lo, b_hi), ...);
}

// R runs 63 down to 0 so that the shifted-in bit of point 64*ib + R lands at
// bit R (of the high word for R >= 32).
template <int MO, int GW, int... Gs>
__device__ __forceinline__ void dom_tile(std::integer_sequence<int, Gs...>,
                                         const NSGA3_RO float *fi, const float (&fj)[MO],
                                         unsigned &a_lo, unsigned &a_hi, unsigned &b_lo,
                                         unsigned &b_hi) {
    constexpr int NG = 64 / GW;
    (dom_group<MO, GW, NG - 1 - Gs>(std::make_integer_sequence<int, GW>{}, fi, fj, a_lo, a_hi,
                                    b_lo, b_hi),
     ...);
}


// Ordered tiles: every column point i is in a lower placement bucket than
// every row point j, so f_1(i) < f_1(j): j cannot dominate i, and
//   i dominates j  <=>  f_i <= f_j in objectives 2 .. m
// (m - 1 compares per column point, no reverse word).
template <int MO, int GW, int R>
__device__ __forceinline__ void dom_step_ord(const ColV<GW> (&v)[MO], const float (&fj)[MO],
                                             unsigned &a_lo, unsigned &a_hi, u64 exec0) {
    u64 le = ~0ull;
    if constexpr (MO >= CMPX_MIN_M) {
        float s[15], w[15];
#pragma unroll
        for (int k = 0; k < 15; ++k) {
            s[k] = k + 1 < MO ? v[k + 1].a[R % GW] : v[1].a[R % GW];
            w[k] = k + 1 < MO ? fj[k + 1] : fj[1];
        }
        le = and_le_exec<MO - 1>(s, w, exec0);
    } else {
#pragma unroll
        for (int k = 1; k < MO; ++k) le &= ballot(v[k].a[R % GW] <= fj[k]);
    }
    if (R >= 32) a_hi = shift_in(a_hi, le);
    else a_lo = shift_in(a_lo, le);
    // keep the step's masks short-lived: unconstrained, the scheduler lifts
    // every compare of the unrolled tile ahead of the shift chain and runs
    // out of scalar registers
    __builtin_amdgcn_sched_barrier(0);
}

// Column values of group g (points GW*g .. GW*g + GW - 1) for objectives
// 2 .. m: one scalar load per objective.
template <int MO, int GW, int g>
__device__ __forceinline__ void load_group_ord(const NSGA3_RO float *fi, ColV<GW> (&v)[MO]) {
#pragma unroll
    for (int k = 1; k < MO; ++k) {
        const NSGA3_RO ColV<GW> &src = *(const NSGA3_RO ColV<GW> *)(fi + k * 64 + GW * g);
#pragma unroll
        for (int q = 0; q < GW; ++q) v[k].a[q] = src.a[q];
    }
}

// Group g of an ordered tile, column points GW*g + GW - 1 down to GW*g, from
// `cur`, while the loads of group g - 1 fill `nxt`. Scalar loads return in
// any order, so a wait for `cur` would also wait for loads issued after it:
// the group waits first, then issues the next group's loads, then computes.
template <int MO, int GW, int g, int... Is>
__device__ __forceinline__ void dom_group_ord(std::integer_sequence<int, Is...>,
                                              const NSGA3_RO float *fi, const float (&fj)[MO],
                                              ColV<GW> (&cur)[MO], ColV<GW> (&nxt)[MO],
                                              unsigned &a_lo, unsigned &a_hi, u64 exec0) {
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (g > 0) load_group_ord<MO, GW, g - 1>(fi, nxt);
    __builtin_amdgcn_sched_barrier(0);
    (dom_step_ord<MO, GW, GW * g + GW - 1 - Is>(cur, fj, a_lo, a_hi, exec0), ...);
#pragma unroll
    for (int k = 1; k < MO; ++k) cur[k] = nxt[k];
}

template <int MO, int GW, int... Gs>
__device__ __forceinline__ void dom_tile_ord(std::integer_sequence<int, Gs...>,
                                             const NSGA3_RO float *fi, const float (&fj)[MO],
                                             unsigned &a_lo, unsigned &a_hi) {
    constexpr int NG = 64 / GW;
    ColV<GW> cur[MO], nxt[MO];
    load_group_ord<MO, GW, NG - 1>(fi, cur);
    const u64 exec0 = __builtin_amdgcn_read_exec();
    (dom_group_ord<MO, GW, NG - 1 - Gs>(std::make_integer_sequence<int, GW>{}, fi, fj, cur, nxt,
                                        a_lo, a_hi, exec0),
     ...);
}

// One wave per work item of the instances with m = MO (the group order[gs ..
// gs + gn)). The item is a run of G consecutive tiles of its instance's
// triangle in row-major order (row jb: column blocks ib = 0 .. jb), so every
// item of an instance carries the same work and one round of waves covers a
// launch. Along a row the 64 points of block jb stay in the lanes (as the
// dominated side j) and the column points of block ib come through the
// scalar cache.
template <int MO>
__global__ __launch_bounds__(256) void k_dominance(BatchView bv, int gs, int gn,
                                                    long long item0, long long n_items) {
    const int lane = lane_id();
    const long long gitem = uniform(item0 + (long long)blockIdx.x * 4 + (threadIdx.x >> 6));
    if (gitem >= item0 + n_items) return;
    const int gi = uniform(find_range(bv.dom_pref + gs, gn, gitem));
    CInst &I = bv.tab[bv.order[gs + gi]];
    const long long item = gitem - bv.dom_pref[gs + gi];
    const int W = I.W, Mp = I.Mp;
    const long long G = I.G, T = tri(W);
    // the objective copy is written by k_prep and only read here: invariant
    // loads, so the column points come through the scalar cache
    const NSGA3_RO float *ft = (const NSGA3_RO float *)I.P.ft;
    u64 *__restrict__ mask = I.P.mask;
    int *__restrict__ nd = I.P.nd;
    const NSGA3_RO int *row_ord = (const NSGA3_RO int *)I.P.row_ord;
    long long t = item * G;
    const long long t_end = t + G < T ? t + G : T;
    int jb = uniform(row_of(t));
    int ib = (int)(t - tri(jb));
    constexpr int GW = col_group<MO>();
    while (t < t_end) {
        const size_t jglob = (size_t)jb * 64 + lane;
        float fj[MO];
#pragma unroll
        for (int k = 0; k < MO; ++k) fj[k] = ft[((size_t)jb * MO + k) * 64 + lane];
        // tiles of this row within the item: the ordered ones first (they
        // write only the row's words), then the rest of the row
        const int ib1 = (int)(t_end - t < (long long)(jb + 1 - ib) ? ib + (t_end - t) : jb + 1);
        const int io = min(ib1, max(ib, uniform(row_ord[jb])));
        int cnt_j = 0;
        for (; ib < io; ++ib) {
            unsigned a_lo = 0, a_hi = 0;
            const NSGA3_RO float *fi = ft + (size_t)ib * MO * 64;
            dom_tile_ord<MO, GW>(std::make_integer_sequence<int, 64 / GW>{}, fi, fj, a_lo, a_hi);
            const u64 A = ((u64)a_hi << 32) | a_lo;
            mask[(size_t)ib * Mp + jglob] = A;
            cnt_j += __popcll(A);
        }
        for (; ib < ib1; ++ib) {
            unsigned a_lo = 0, a_hi = 0, b_lo = 0, b_hi = 0;
            const NSGA3_RO float *fi = ft + (size_t)ib * MO * 64;
            dom_tile<MO, GW>(std::make_integer_sequence<int, 64 / GW>{}, fi, fj, a_lo, a_hi, b_lo,
                             b_hi);
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
        t = tri(jb) + ib1;
        ++jb;
        ib = 0;
    }
}

// Dominance for m > NARROW_M (the many-objective regime): the objectives of a
// point no longer fit in registers, so each tile runs over chunks of DW_KC
// objectives. Per chunk, the wave stages the column block's values in LDS
// (its own region) and keeps the row values in registers; per column point i
// it ORs the ballots lt_i = {j : f_i < f_j in some objective} and gt_i =
// {j : f_i > f_j in some objective} into per-wave LDS words. A column point
// whose every row point is already incomparable (lt_i and gt_i both set) is
// skipped, and the tile ends once every column point is, which at large m
// comes after a few objectives for most pairs. The words are those of
// k_dominance: bit i of row word j is i -> j (j in lt_i \ gt_i), and column
// point i's word from this row block is gt_i \ lt_i. Work items, tiles and
// the fused counts are as in k_dominance.
constexpr int DW_KC = 32;

__global__ __launch_bounds__(256) void k_dominance_wide(BatchView bv, int gs, int gn,
                                                         long long item0, long long n_items) {
    __shared__ float s_col[4][64][DW_KC + 1];  // padded rows: conflict-free staging
    __shared__ u64 s_lt[4][64], s_gt[4][64];
    const int lane = lane_id();
    const int wv = threadIdx.x >> 6;
    const long long gitem = uniform(item0 + (long long)blockIdx.x * 4 + wv);
    if (gitem >= item0 + n_items) return;
    const int gi = uniform(find_range(bv.dom_pref + gs, gn, gitem));
    CInst &I = bv.tab[bv.order[gs + gi]];
    const long long item = gitem - bv.dom_pref[gs + gi];
    const int W = I.W, Mp = I.Mp, m = I.m, M = I.M;
    const long long G = I.G, T = tri(W);
    const float *__restrict__ ft = I.P.ft;
    u64 *__restrict__ mask = I.P.mask;
    int *__restrict__ nd = I.P.nd;
    long long t = item * G;
    const long long t_end = t + G < T ? t + G : T;
    while (t < t_end) {
        const int jb = uniform(row_of(t));
        const int ib = (int)(t - tri(jb));
        const u64 rowvalid = M - jb * 64 >= 64 ? ~0ull : ((1ull << (M - jb * 64)) - 1);
        const int ncol = M - ib * 64 >= 64 ? 64 : M - ib * 64;  // real column points
        s_lt[wv][lane] = 0ull;
        s_gt[wv][lane] = 0ull;
        for (int k0 = 0; k0 < m; k0 += DW_KC) {
            const int kc = m - k0 < DW_KC ? m - k0 : DW_KC;
            float fj[DW_KC];
#pragma unroll
            for (int kk = 0; kk < DW_KC; ++kk) {
                fj[kk] = kk < kc ? ft[((size_t)jb * m + k0 + kk) * 64 + lane] : 0.0f;
                if (kk < kc) s_col[wv][lane][kk] = ft[((size_t)ib * m + k0 + kk) * 64 + lane];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            int open = 0;
            for (int i = 0; i < ncol; ++i) {
                u64 lt = uniform(s_lt[wv][i]), gt = uniform(s_gt[wv][i]);
                if (((lt & gt) | ~rowvalid) == ~0ull) continue;
                for (int kk = 0; kk < kc; ++kk) {
                    const float x = s_col[wv][i][kk];
                    lt |= ballot(x < fj[kk]);
                    gt |= ballot(x > fj[kk]);
                }
                if (lane == 0) {
                    s_lt[wv][i] = lt;
                    s_gt[wv][i] = gt;
                }
                open += ((lt & gt) | ~rowvalid) != ~0ull;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (uniform(open) == 0) break;  // every pair of the tile is incomparable
        }
        // row word of lane j: bit i = i -> j
        u64 A = 0;
        for (int i = 0; i < ncol; ++i) {
            const u64 d = uniform(s_lt[wv][i]) & ~uniform(s_gt[wv][i]);
            A |= ((d >> lane) & 1ull) << i;
        }
        mask[(size_t)ib * Mp + (size_t)jb * 64 + lane] = A;
        const int cnt_j = __popcll(A);
        if (cnt_j) atomicAdd(&nd[jb * 64 + lane], cnt_j);
        if (ib != jb) {
            // column point i = lane: its dominators in row block jb
            const u64 B = lane < ncol ? (s_gt[wv][lane] & ~s_lt[wv][lane] & rowvalid) : 0ull;
            mask[(size_t)jb * Mp + (size_t)ib * 64 + lane] = B;
            const int c = __popcll(B);
            if (c) atomicAdd(&nd[ib * 64 + lane], c);
        }
        __builtin_amdgcn_wave_barrier();  // LDS words are reused by the next tile
        ++t;
    }
}

// Front peeling.
//
// Chunk c of an instance holds its 64 points 64c .. 64c+63. Every point keeps
// the number of its dominators that are still alive (not yet ranked), starting
// from the fused counts of the dominance kernel; front k is the set of alive
// points whose count is zero. When front k - 1 is known, each chunk subtracts,
// for every block w of 64 points that lost members to front k - 1, the
// popcount of (its points' word w of the dominance matrix) AND (those
// members), no per-point searching. The matrix words of a chunk are either
// held in registers from front 1 on (load_column) or streamed, one coalesced
// 512-byte load per block w and wave, all blocks in flight at once. The peel
// of an instance stops once its ranked fronts hold n_stop points.
//
// Scheduling. While ranking front 0, workgroups claim chunks (of any
// instance) from sharded ticket counters until every chunk is claimed; a
// workgroup then owns its chunks for all later fronts and processes them
// front by front. Only running workgroups claim, and no workgroup waits
// before all chunks are claimed and ranked for front 0; later waits are for
// lower fronts of chunks owned by running workgroups, so every wait ends. A
// workgroup records at most PEEL_OWN_CAP chunks; if every running workgroup
// were full the front-1 wait would time out into an error status.
//
// Publication. When chunk c has ranked its members of front k, it stores them
// in slot k % PEEL_RING of the instance's front ring as two tagged words (the
// tag k + 1 in the high 32 bits; the low, then the high 32 bits of the member
// mask in the low 32 bits), and waits for nothing. A workgroup waiting for
// front k polls all tagged words of the slot: once every tag reads k + 1, the
// same loads have delivered the members of front k of every block, and their
// popcounts give the front's size. A slot is written again (for front
// k + PEEL_RING) only after front k + PEEL_RING - 1 completed, which needs every
// owner to have read front k before; the tag tells a stale word from a
// current one, and the ring is zeroed when the call starts, so no word of an
// earlier call carries a current tag.
//
// Memory ordering. Tagged words are written with agent-scope atomic stores
// and polled with agent-scope atomic loads, so every read sees the coherent
// level; an aligned 64-bit store is single-copy atomic, so a word with a
// current tag carries its current half of the mask. A chunk's counts and its
// alive mask are read and written only by wave 0 of its owner.
//
// Control flow is wave-uniform around every workgroup barrier: wave 0 makes
// the scheduling decisions with all its lanes and shares them through LDS.
// Consecutive owned chunks of one instance share one wait, so no barrier
// separates wave 0's update of a chunk's running total from the other waves'
// read of it; the totals are therefore kept twice, by the parity of the
// front, and a wave never reads a value written for the front after.
// Barriers order LDS only (they do not wait for global stores in flight).
constexpr int PEEL_WAVES = 8;
constexpr int PEEL_OWN_CAP = 1024;
constexpr int PEEL_LDS_ALIVE = 2048;  // blocks whose members are staged in LDS (M <= 131072)
constexpr int PEEL_BATCH = 16;        // matrix loads in flight per wave (streamed columns)
constexpr int PEEL_CACHE_SLOTS = 2;   // owned chunks whose columns stay in registers
constexpr unsigned PEEL_POLLS = 1u << 22;  // polls of one word before a wait gives up (an internal error)

// Tagged members of front k: slot k % PEEL_RING of the ring (2W words,
// padded to whole 128-byte lines).
__device__ __forceinline__ u64 *front_slot(u64 *ring, int W, int k) {
    return ring + (size_t)(k % PEEL_RING) * front_slot_words(W);
}

struct PeelShared {
    int own_b[PEEL_OWN_CAP];    // instance of each owned chunk
    int own_c[PEEL_OWN_CAP];    // chunk within its instance
    // points in the instance's fronts before front k - 1 (-1: done), read
    // from [k & 1] and written to [(k + 1) & 1] while front k is processed
    int own_cum[2][PEEL_OWN_CAP];
    u64 own_alive[PEEL_OWN_CAP];  // its points not yet ranked
    u64 dead[PEEL_LDS_ALIVE];   // members of the awaited front, per block of 64 points
    int part[PEEL_CACHE_SLOTS][PEEL_WAVES][64];  // per-wave partial decrements of a chunk's counts
    int cleft[PEEL_CACHE_SLOTS][64];  // counts of the cached chunks
    int red_bad[PEEL_WAVES];    // per-wave poll results
    int red_cnt[PEEL_WAVES];
    u64 val, val2;
};

// Members of front kf in block w, from the tagged words (current tags
// verified by the wait).
__device__ __forceinline__ u64 tagged_members(const u64 *slot, int w) {
    const u64 lo = load_relaxed(&slot[2 * w]), hi = load_relaxed(&slot[2 * w + 1]);
    return (lo & 0xffffffffull) | (hi << 32);
}

// Waits until every chunk of I has published front kf; stages its members
// in LDS when STAGED. Returns the front's size, or -1 if a wait gave up.
// Every thread polls its own words until their tags are current, so the
// workgroup meets once, when all are. All waves take part.
template <bool STAGED>
__device__ int await_front(const CInst &I, int kf, PeelShared &sh) {
    const int W = I.W;
    const int wv = uniform((int)(threadIdx.x >> 6));
    const u64 *slot = front_slot(I.P.ring, W, kf);
    const unsigned tag = (unsigned)kf + 1u;
    bool bad = false;
    int cnt = 0;
    for (int w = threadIdx.x; w < W; w += blockDim.x) {
        u64 lo, hi;
        for (unsigned polls = 0;; ++polls) {
            lo = load_relaxed(&slot[2 * w]);
            hi = load_relaxed(&slot[2 * w + 1]);
            if ((unsigned)(lo >> 32) == tag && (unsigned)(hi >> 32) == tag) break;
            if (polls == PEEL_POLLS) {
                bad = true;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        const u64 d = (lo & 0xffffffffull) | (hi << 32);
        cnt += __popcll(d);
        if (STAGED) sh.dead[w] = d;
    }
    const int wbad = ballot(bad) != 0;
    const int wcnt = wave_sum(cnt);
    if (lane_id() == 0) {
        sh.red_bad[wv] = wbad;
        sh.red_cnt[wv] = wcnt;
    }
    lds_barrier();
    int anybad = 0, total = 0;
#pragma unroll
    for (int v = 0; v < PEEL_WAVES; ++v) {
        anybad |= sh.red_bad[v];
        total += sh.red_cnt[v];
    }
    anybad = uniform(anybad);
    total = uniform(total);
    lds_barrier();  // the shared words may be overwritten after this
    return anybad ? -1 : total;
}

// Column cache of an owned chunk c: its matrix words mask[w * Mp + 64c +
// lane] for w = wv + q * PEEL_WAVES (q < Q), zero from w = W on, loaded once
// and held in registers for every later front (the matrix is then read once
// per chunk instead of once per front).
template <int Q>
__device__ __forceinline__ void load_column(const CInst &I, int c, u64 (&col)[Q]) {
    const int wv = uniform((int)(threadIdx.x >> 6));
    const u64 *p = I.P.mask + (size_t)c * 64 + lane_id();
    const int we = uniform(I.P.col_end[c]);  // zero (and unwritten) from here on
    const size_t Mp = (size_t)I.Mp;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int w = wv + q * PEEL_WAVES;
        col[q] = w < we ? p[(size_t)w * Mp] : 0ull;
    }
}

// Publishes the members `newly` of front k in chunk c (one wave; lanes 0 and
// 1 store the tagged halves) and records the chunk's remaining points.
__device__ __forceinline__ void publish(CInst &I, int k, int c, int own, u64 aw, u64 newly,
                                        PeelShared &sh) {
    const int lane = lane_id();
    if (lane < 2) {
        const u64 tag = (u64)(k + 1) << 32;
        const u64 half = lane == 0 ? (newly & 0xffffffffull) : (newly >> 32);
        store_relaxed(&front_slot(I.P.ring, I.W, k)[2 * c + lane], tag | half);
    }
    if (lane == 0) sh.own_alive[own] = aw & ~newly;
    if ((newly >> lane) & 1ull) I.rank[I.P.perm[c * 64 + lane]] = k;  // read only by later kernels
}

// Ranks the points of owned chunk `own` (chunk c of I) that are alive at
// front k and have no alive dominator, and publishes them. For k > 0 the
// members of front k - 1 are those of the last await_front on I (staged in
// LDS when STAGED, W <= PEEL_LDS_ALIVE; a compile-time choice, so that no
// pointer ever selects between LDS and global memory). Q > 0: the chunk's
// column is in `col` and its counts in sh.cleft[own] (needs STAGED and W <=
// Q * PEEL_WAVES); Q = 0: its counts are in nd and its column is streamed,
// BATCH loads in flight per wave. All waves take part.
template <bool STAGED, int Q, int BATCH>
__device__ void peel_chunk_impl(CInst &I, int k, int c, int own, PeelShared &sh,
                                const u64 (&col)[Q > 0 ? Q : 1]) {
    const int lane = lane_id();
    const int wv = uniform((int)(threadIdx.x >> 6));
    const int W = I.W;
    const int j = c * 64 + lane;
    int *nd = I.P.nd;
    u64 aw, newly;
    if (k == 0) {
        const int valid = I.M - c * 64;
        aw = valid >= 64 ? ~0ull : ((1ull << valid) - 1);
        newly = aw & ballot(nd[j] == 0);
    } else {
        aw = uniform(sh.own_alive[own]);
        int left = 0;  // alive dominators before front k - 1 is removed
        if (wv == 0) {
            if constexpr (Q > 0) left = sh.cleft[own][lane];
            else left = nd[j];
        }
        if (aw != 0) {
            // wave wv takes blocks wv, wv + PEEL_WAVES, ...
            int acc = 0;
            if constexpr (Q > 0) {
                // words from w = W on are zero in the cache
#pragma unroll
                for (int q = 0; q < Q; ++q) acc += __popcll(col[q] & sh.dead[wv + q * PEEL_WAVES]);
            } else {
                const u64 *__restrict__ src = I.P.mask + (size_t)c * 64 + lane;
                const u64 *slot = front_slot(I.P.ring, W, k - 1);
                const size_t Mp = (size_t)I.Mp;
                const int we = uniform(I.P.col_end[c]);  // zero words from here on
                for (int w0 = wv; w0 < we; w0 += PEEL_WAVES * BATCH) {
                    u64 x[BATCH], d[BATCH];
#pragma unroll
                    for (int q = 0; q < BATCH; ++q) {
                        const int w = w0 + q * PEEL_WAVES;
                        d[q] = w < we ? (STAGED ? sh.dead[w] : tagged_members(slot, w)) : 0ull;
                        x[q] = d[q] ? src[(size_t)w * Mp] : 0ull;
                    }
#pragma unroll
                    for (int q = 0; q < BATCH; ++q) acc += __popcll(x[q] & d[q]);
                }
            }
            sh.part[0][wv][lane] = acc;
        }
        lds_barrier();
        newly = 0;
        if (wv == 0 && aw != 0) {
#pragma unroll
            for (int v = 0; v < PEEL_WAVES; ++v) left -= sh.part[0][v][lane];
            const bool alive = (aw >> lane) & 1ull;
            if (alive) {
                if constexpr (Q > 0) sh.cleft[own][lane] = left;
                else nd[j] = left;
            }
            newly = aw & ballot(alive && left == 0);
        }
        lds_barrier();  // the shared partial sums are free again
    }
    if (wv == 0) publish(I, k, c, own, aw, newly, sh);
}

// Both cached chunks (c0, c1: owned slots 0 and 1 of the same instance) in
// one pass for front k >= 1: every wave sweeps its blocks for both columns,
// then wave s finishes chunk s.
template <int Q>
__device__ void peel_pair(CInst &I, int k, int c0, int c1, PeelShared &sh, const u64 (&col0)[Q],
                          const u64 (&col1)[Q]) {
    const int lane = lane_id();
    const int wv = uniform((int)(threadIdx.x >> 6));
    int acc0 = 0, acc1 = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const u64 d = sh.dead[wv + q * PEEL_WAVES];
        acc0 += __popcll(col0[q] & d);
        acc1 += __popcll(col1[q] & d);
    }
    sh.part[0][wv][lane] = acc0;
    sh.part[1][wv][lane] = acc1;
    lds_barrier();
    if (wv < 2) {
        const int s = wv;
        const u64 aw = uniform(sh.own_alive[s]);
        int left = sh.cleft[s][lane];
#pragma unroll
        for (int v = 0; v < PEEL_WAVES; ++v) left -= sh.part[s][v][lane];
        const bool alive = (aw >> lane) & 1ull;
        if (alive) sh.cleft[s][lane] = left;
        const u64 newly = aw & ballot(alive && left == 0);
        publish(I, k, s ? c1 : c0, s, aw, newly, sh);
    }
    lds_barrier();  // the shared partial sums are free again
}

// A chunk whose column is streamed.
template <int BATCH>
__device__ __forceinline__ void peel_chunk(CInst &I, int k, int c, int own, PeelShared &sh) {
    const u64 none[1] = {0ull};
    if (uniform(I.W) <= PEEL_LDS_ALIVE) peel_chunk_impl<true, 0, BATCH>(I, k, c, own, sh, none);
    else peel_chunk_impl<false, 0, BATCH>(I, k, c, own, sh, none);
}

// Q > 0: the first PEEL_CACHE_SLOTS chunks a workgroup owns keep their
// columns in registers (every instance has W <= Q * PEEL_WAVES); further
// chunks, if any, are streamed. The launch peels chunks c0 .. c0 + nchunk - 1
// of the batch's chunk order (whole m-groups) and claims them from word tw
// of each ticket shard.
template <int Q>
__global__ __launch_bounds__(64 * PEEL_WAVES) void k_peel(BatchView bv, int c0, int nchunk,
                                                         int tw) {
    constexpr int BATCH = Q > 0 ? 4 : PEEL_BATCH;  // streamed chunks: fewer registers next to a cache
    __shared__ PeelShared sh;
    const int lane = lane_id();
    const int wv = uniform((int)(threadIdx.x >> 6));

    // Front 0: claim chunks until all are claimed. Ticket shard s hands out
    // chunks s, s + TICKET_SHARDS, ...; a workgroup starts at its own shard
    // and moves on when one runs dry (the shards spread the claims over many
    // addresses). One atomic claims up to `take` (1 or 2) chunks: tickets n
    // and n + 1 of a shard. Returns the first claimed chunk (uniform; nchunk
    // or more when none is left) and the second in t2 (nchunk or more when
    // there is none).
    int nown = 0;
    const int home = (int)(blockIdx.x % TICKET_SHARDS);
    bool home_dry = false;
    auto claim = [&](int take, u64 &t2) -> u64 {
        if (wv == 0) {
            const u64 add = lane == 0 ? (u64)take : 0ull;
            u64 t = ~0ull, u = ~0ull;
            for (;;) {
                int s = home;
                if (home_dry) {
                    // look at every shard at once; claim from one that has
                    // chunks left (starting after the home shard), or stop
                    // when none has
                    const u64 n_l = lane < TICKET_SHARDS
                                        ? load_relaxed(&bv.ticket[lane * TICKET_STRIDE + tw])
                                        : 0ull;
                    const u64 avail = ballot(lane < TICKET_SHARDS &&
                                             (u64)lane + (u64)TICKET_SHARDS * n_l < (u64)nchunk);
                    if (avail == 0) break;
                    // the 32 shard bits rotated so that the home shard is bit 0
                    const unsigned a32 = (unsigned)avail;
                    const unsigned rot = home == 0 ? a32 : ((a32 >> home) | (a32 << (32 - home)));
                    s = (home + __ffs((int)rot) - 1) % TICKET_SHARDS;
                }
                const u64 n = uniform(atomicAdd(&bv.ticket[s * TICKET_STRIDE + tw], add));
                const u64 g = (u64)s + (u64)TICKET_SHARDS * n;
                // the shard's next ticket after these is past the end: dry
                if (s == home && g + (u64)TICKET_SHARDS * (u64)take >= (u64)nchunk) home_dry = true;
                if (g < (u64)nchunk) {
                    t = g;
                    if (take > 1 && g + TICKET_SHARDS < (u64)nchunk) u = g + TICKET_SHARDS;
                    break;
                }
            }
            sh.val = t;
            sh.val2 = u;
        }
        lds_barrier();
        const u64 t = uniform(sh.val);
        t2 = uniform(sh.val2);
        lds_barrier();
        return t;
    };
    // Records claimed chunk t as owned chunk nown (wave 0 writes, the
    // caller's next barrier publishes it).
    auto own = [&](u64 t, int &b, int &c) {
        const int tt = c0 + (int)t;
        const int pos = uniform(find_range(bv.chunk_pref, bv.B, tt));
        b = uniform(bv.order[pos]);
        c = tt - bv.chunk_pref[pos];
        if (wv == 0) {
            sh.own_b[nown] = b;
            sh.own_c[nown] = c;
            sh.own_cum[1][nown] = 0;
        }
    };
    // Front 0 of every chunk comes from the counts fused into the dominance
    // kernel. Streamed columns: front 0 of each chunk at its claim. Cached
    // columns: up to PEEL_CACHE_SLOTS claims, front 0 of those, then their
    // column loads; then, while chunks are left, further claims streamed as
    // above. Every running workgroup claims until none is left, so every
    // chunk has a running owner.
    bool dry = false;
    constexpr int FIRST_CAP = Q > 0 ? PEEL_CACHE_SLOTS : PEEL_OWN_CAP;
    while (nown < FIRST_CAP) {
        u64 t2;
        const u64 t = claim(FIRST_CAP - nown >= 2 ? 2 : 1, t2);
        if (t >= (u64)nchunk) { dry = true; break; }
        for (u64 tc : {t, t2}) {
            if (tc >= (u64)nchunk) break;
            int b, c;
            own(tc, b, c);
            if (Q == 0) peel_chunk<BATCH>(bv.tab[b], 0, c, nown, sh);
            ++nown;
        }
    }
    lds_barrier();
    u64 col0[Q > 0 ? Q : 1], col1[Q > 0 ? Q : 1];
    if constexpr (Q > 0) {
        if (nown > 0) {
            // front 0 of the cached chunks from the counts fused into the
            // dominance kernel, published before their columns arrive (the
            // loads overlap the wait for the other chunks' front 0)
            if (wv < nown) {  // waves 0 and 1: slots 0 and 1
                const int slot = wv;
                CInst &I = bv.tab[uniform(sh.own_b[slot])];
                const int c = uniform(sh.own_c[slot]);
                const int cnt = I.P.nd[c * 64 + lane];
                sh.cleft[slot][lane] = cnt;
                const int valid = I.M - c * 64;
                const u64 aw = valid >= 64 ? ~0ull : ((1ull << valid) - 1);
                publish(I, 0, c, slot, aw, aw & ballot(cnt == 0), sh);
            }
        }
        // Are chunks left to claim? Wave 0 reads the shard counters (one
        // round trip) before its column loads, so waiting for them does not
        // wait for the columns, and the check overlaps the loads.
        u64 n_l = 0;
        if (!dry && wv == 0 && lane < TICKET_SHARDS)
            n_l = load_relaxed(&bv.ticket[lane * TICKET_STRIDE + tw]);
        if (nown > 0) {
            const int b0 = uniform(sh.own_b[0]), c0 = uniform(sh.own_c[0]);
            load_column<Q>(bv.tab[b0], c0, col0);
            if (nown > 1) load_column<Q>(bv.tab[uniform(sh.own_b[1])], uniform(sh.own_c[1]), col1);
        }
        if (!dry && wv == 0) {
            const u64 avail = ballot(lane < TICKET_SHARDS &&
                                     (u64)lane + (u64)TICKET_SHARDS * n_l < (u64)nchunk);
            if (lane == 0) sh.val2 = avail;
        }
        lds_barrier();  // the published state and the check are visible to every wave
        // (counters only grow: when no shard has a ticket left, every chunk
        // has an owner)
        if (!dry && uniform(sh.val2) == 0) dry = true;
        // chunks beyond the cache slots: streamed, front 0 at the claim
        while (!dry && nown < PEEL_OWN_CAP) {
            u64 t2;
            const u64 t = claim(PEEL_OWN_CAP - nown >= 2 ? 2 : 1, t2);
            if (t >= (u64)nchunk) break;
            for (u64 tc : {t, t2}) {
                if (tc >= (u64)nchunk) break;
                int b, c;
                own(tc, b, c);
                peel_chunk<BATCH>(bv.tab[b], 0, c, nown, sh);
                ++nown;
            }
        }
        lds_barrier();
    }
    // a workgroup without chunks has nothing left to do; the owners of the
    // chunks report the front fill
    if (nown == 0) return;

    for (int k = 1;; ++k) {
        const int cur = k & 1, nxt = cur ^ 1;
        int active = 0;
        int awaited = -1, size = 0;  // instance whose front k - 1 was last awaited
        for (int q = 0; q < nown; ++q) {
            const int b = uniform(sh.own_b[q]);
            const int c = uniform(sh.own_c[q]);
            const int cum_prev = uniform(sh.own_cum[cur][q]);
            if (cum_prev < 0) {  // this instance finished
                if (wv == 0) sh.own_cum[nxt][q] = -1;
                continue;
            }
            CInst &I = bv.tab[b];
            const bool staged = uniform(I.W) <= PEEL_LDS_ALIVE;
            // wait for front k - 1 of the instance (already staged when the
            // previous owned chunk belongs to the same instance)
            if (b != awaited) {
                size = staged ? await_front<true>(I, k - 1, sh) : await_front<false>(I, k - 1, sh);
                awaited = b;
            }
            const int cum = cum_prev + size;
            if (size <= 0 || cum >= I.n_stop) {
                if (wv == 0) {
                    if (size <= 0) atomicOr(&I.P.ctrl->status, ST_INTERNAL);
                    I.front_info[0] = k - 1;
                    I.front_info[1] = cum_prev;
                    I.front_info[2] = I.n_stop - cum_prev;
                    I.front_info[3] = k;
                    sh.own_cum[nxt][q] = -1;
                }
                continue;
            }
            if (wv == 0) sh.own_cum[nxt][q] = cum;
            if constexpr (Q > 0) {
                static_assert(PEEL_CACHE_SLOTS == 2, "one branch per cached slot");
                // both cached chunks of one instance, together
                if (q == 0 && nown > 1 && uniform(sh.own_b[1]) == b && uniform(sh.own_cum[cur][1]) >= 0) {
                    if (wv == 0) sh.own_cum[nxt][1] = cum;
                    peel_pair<Q>(I, k, c, uniform(sh.own_c[1]), sh, col0, col1);
                    active = 1;
                    q = 1;
                    continue;
                }
                if (q == 0) peel_chunk_impl<true, Q, BATCH>(I, k, c, q, sh, col0);
                else if (q == 1) peel_chunk_impl<true, Q, BATCH>(I, k, c, q, sh, col1);
                else peel_chunk<BATCH>(I, k, c, q, sh);
            } else {
                peel_chunk<BATCH>(I, k, c, q, sh);
            }
            active = 1;
        }
        lds_barrier();
        if (!active) break;
    }
}

hipError_t launch_prepare(const HostPlan &hp, const BatchView &bv, bool init_done, hipStream_t s) {
    if (!init_done) NSGA3_LAUNCH("init", k_init, dim3(hp.B), dim3(256), 0, s, bv);
    NSGA3_LAUNCH("prep", k_prep, dim3((hp.npt + hp.nref) / 256), dim3(256), 0, s, bv, hp.npt);
    if (bv.run & RUN_ND) {
        // the objective copy by scattered stores while it fits the L2, else
        // by a gather in position order
        const long long copy_bytes = (long long)hp.npt * hp.grp_m[hp.ngroups - 1] * 4;
        const int scatter = copy_bytes <= PLACE_SCATTER_BYTES ? 1 : 0;
        NSGA3_LAUNCH("place_scatter", k_place_scatter, dim3(hp.npt / 256), dim3(256), 0, s, bv,
                     scatter);
        if (!scatter)
            NSGA3_LAUNCH("place_gather", k_place_gather, dim3(hp.npt / 256), dim3(256), 0, s, bv);
    }
    return hipGetLastError();
}

// Column caching of a peel over `nchunk` chunks whose widest instance has
// W = max_W: columns stay in registers (returns the per-wave cache size) when
// every column fits a cache and two cached chunks per compute unit hold all
// chunks (one workgroup per compute unit at that register use); otherwise
// they are streamed (returns 0). Either way front 0 comes from the counts
// fused into the dominance kernel (no pass over the matrix before it).
static int peel_cache(int nchunk, int max_W, int cus) {
    if (nchunk > PEEL_CACHE_SLOTS * cus) return 0;
    for (int c : {16, 24, 32, 40, 48})
        if (max_W <= c * PEEL_WAVES) return c;
    return 0;
}

// Workgroups of a peel: one per compute unit with cached columns (their
// register use), else `streamed_per_cu` per compute unit.
static void launch_peel(const BatchView &bv, int q, int c0, int nchunk, int tw, int cus,
                        int streamed_per_cu, hipStream_t s) {
    const int cap = q ? cus : streamed_per_cu * cus;
    const dim3 pg(nchunk < cap ? nchunk : cap), pb(64 * PEEL_WAVES);
    switch (q) {
        case 16: NSGA3_LAUNCH("peel", k_peel<16>, pg, pb, 0, s, bv, c0, nchunk, tw); break;
        case 24: NSGA3_LAUNCH("peel", k_peel<24>, pg, pb, 0, s, bv, c0, nchunk, tw); break;
        case 32: NSGA3_LAUNCH("peel", k_peel<32>, pg, pb, 0, s, bv, c0, nchunk, tw); break;
        case 40: NSGA3_LAUNCH("peel", k_peel<40>, pg, pb, 0, s, bv, c0, nchunk, tw); break;
        case 48: NSGA3_LAUNCH("peel", k_peel<48>, pg, pb, 0, s, bv, c0, nchunk, tw); break;
        default: NSGA3_LAUNCH("peel", k_peel<0>, pg, pb, 0, s, bv, c0, nchunk, tw); break;
    }
}

static void launch_dominance(const HostPlan &hp, const BatchView &bv, int g, hipStream_t s) {
    const int gs = hp.grp_start[g], gn = hp.grp_start[g + 1] - gs;
    const long long item0 = hp.grp_dom[g], n_items = hp.grp_dom[g + 1] - item0;
    const unsigned blocks = (unsigned)((n_items + 3) / 4);
#define NSGA3_DOM_CASE(MO)                                                                       \
    case MO:                                                                                     \
        NSGA3_LAUNCH("dominance", k_dominance<MO>, dim3(blocks), dim3(256), 0, s, bv, gs, gn,   \
                     item0, n_items);                                                            \
        break;
    switch (hp.grp_m[g]) {
        NSGA3_DOM_CASE(2) NSGA3_DOM_CASE(3) NSGA3_DOM_CASE(4) NSGA3_DOM_CASE(5)
        NSGA3_DOM_CASE(6) NSGA3_DOM_CASE(7) NSGA3_DOM_CASE(8) NSGA3_DOM_CASE(9)
        NSGA3_DOM_CASE(10) NSGA3_DOM_CASE(11) NSGA3_DOM_CASE(12) NSGA3_DOM_CASE(13)
        NSGA3_DOM_CASE(14) NSGA3_DOM_CASE(15) NSGA3_DOM_CASE(16)
        default:
            NSGA3_LAUNCH("dominance", k_dominance_wide, dim3(blocks), dim3(256), 0, s, bv, gs, gn,
                         item0, n_items);
            break;
    }
#undef NSGA3_DOM_CASE
}

// Pipelined peel of a batch with several m-groups: each group's peel runs on
// a side stream as soon as that group's dominance launch is done, beside the
// dominance launches of the later groups (the peel is bound by the latency of
// its fronts, the dominance by vector issue). The side stream forks from the
// caller's stream and joins it again through events, so the call stays one
// ordered piece of work on the caller's stream and can be captured in a
// graph. One side stream and event set per device, made on the first batched
// call outside a capture and kept until the process ends; a mutex orders
// their use by calls from several host threads.
// Workgroups per compute unit of a streamed peel beside dominance launches
// (the rest of each compute unit's wave slots stay with the dominance).
constexpr int PEEL_PIPE_PER_CU = 1;

struct PeelPipe {
    hipStream_t side = nullptr;
    hipEvent_t ev[PEEL_PIPE_GROUPS + 1] = {};
};
static std::mutex g_pipe_mu;
static PeelPipe g_pipe[64];

static unsigned long long capture_id(hipStream_t s, bool &capturing, bool &ok) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    unsigned long long id = 0;
    ok = hipStreamGetCaptureInfo(s, &st, &id) == hipSuccess &&
         st != hipStreamCaptureStatusInvalidated;
    capturing = st == hipStreamCaptureStatusActive;
    return id;
}

// The device's pipe if the peel may be pipelined now, else null (the caller
// then peels in one launch): the pipe is made outside a capture only, and its
// side stream must be idle in capture terms or in the caller's own capture.
static PeelPipe *pipe_for(hipStream_t s) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    bool cap_s, ok_s;
    const unsigned long long id_s = capture_id(s, cap_s, ok_s);
    if (!ok_s) return nullptr;
    PeelPipe &p = g_pipe[dev];
    if (!p.side) {
        if (cap_s) return nullptr;
        hipStream_t side;
        if (hipStreamCreateWithFlags(&side, hipStreamNonBlocking) != hipSuccess) return nullptr;
        for (int i = 0; i <= PEEL_PIPE_GROUPS; ++i)
            if (hipEventCreateWithFlags(&p.ev[i], hipEventDisableTiming) != hipSuccess) {
                for (int k = 0; k < i; ++k) (void)hipEventDestroy(p.ev[k]);
                (void)hipStreamDestroy(side);
                return nullptr;
            }
        p.side = side;
    }
    bool cap_side, ok_side;
    const unsigned long long id_side = capture_id(p.side, cap_side, ok_side);
    if (!ok_side || (cap_side && (!cap_s || id_side != id_s))) return nullptr;
    return &p;
}

hipError_t launch_nd_sort(const HostPlan &hp, const BatchView &bv, hipStream_t s, bool *through) {
    const int cus = device_info().cus;
    if (hp.B > 1 && hp.ngroups > 1 && hp.ngroups <= PEEL_PIPE_GROUPS) {
        std::lock_guard<std::mutex> lock(g_pipe_mu);
        if (PeelPipe *p = pipe_for(s)) {
            hipError_t e = hipSuccess;
            for (int g = 0; g < hp.ngroups && e == hipSuccess; ++g) {
                const int c0 = hp.grp_chunk[g], nc = hp.grp_chunk[g + 1] - c0;
                const int q = peel_cache(nc, hp.grp_max_W[g], cus);
                launch_dominance(hp, bv, g, s);
                e = hipEventRecord(p->ev[g], s);
                if (e == hipSuccess) e = hipStreamWaitEvent(p->side, p->ev[g], 0);
                if (e == hipSuccess) {
                    launch_peel(bv, q, c0, nc, g, cus, PEEL_PIPE_PER_CU, p->side);
                    // the group's normalization and association sweep need
                    // only its own ranks (their grids skip other groups)
                    if (*through) {
                        launch_norm_fused_group(hp, bv, g, p->side);
                        launch_associate_group(hp, bv, g, p->side);
                    }
                }
            }
            // join even after an error, so that the side stream leaves no
            // open fork in a capture
            const hipError_t ej = hipEventRecord(p->ev[PEEL_PIPE_GROUPS], p->side);
            const hipError_t ew = ej == hipSuccess
                                      ? hipStreamWaitEvent(s, p->ev[PEEL_PIPE_GROUPS], 0)
                                      : ej;
            if (e == hipSuccess) e = ew;
            return e == hipSuccess ? hipGetLastError() : e;
        }
    }
    *through = false;
    const int q = peel_cache(hp.nchunk, hp.max_W, cus);
    for (int g = 0; g < hp.ngroups; ++g) launch_dominance(hp, bv, g, s);
    launch_peel(bv, q, 0, hp.nchunk, 0, cus, 3, s);
    return hipGetLastError();
}

}  // namespace nsga3
