/*
 * CPU oracle for NSGA-III environmental selection (TEST INFRASTRUCTURE ONLY).
 *
 * This library is the slow, obviously-correct FP64 definition that the GPU
 * path is checked against. Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it. It shares no code with the HIP
 * library: no headers, no helpers, no tables.
 *
 * Method: NSGA-III selection as stated in the paper (Sec. II-C, Algorithm 1;
 * tensorized restatement in Sec. III-B, Algorithm 2 and Eq. 1), with the
 * normalization of Deb & Jain 2014 (the NSGA-III reference cited in Sec. II-C)
 * and random tie-breaks replaced by a SplitMix64-keyed deterministic rule.
 *
 * Conventions shared with the GPU path (they are part of the specification,
 * not of either implementation):
 *   - objectives are minimized; F is row-major [M][m] float32;
 *   - ranks are 0-based; points in fronts after the last selected front carry
 *     ORACLE_UNRANKED;
 *   - front_info = {l, |S|, K, l + 1} with l the 0-based index of the
 *     last (partially selected) front, S the fully selected fronts, and
 *     K = N - |S| the number of picks made from front l;
 *   - selected[] is the ascending list of the N chosen indices.
 *
 * Every entry point returns 0 on success and a negative code on bad arguments.
 */
#ifndef NSGA3_ORACLE_H
#define NSGA3_ORACLE_H
#include <stdint.h>

#define ORACLE_UNRANKED 0x7fffffff
#define ORACLE_MAX_OBJECTIVES 512

#ifdef __cplusplus
extern "C" {
#endif

/* Threads used by the dominance and association loops (default 1, the plain
 * serial loops). Results do not depend on it. Returns the count set. */
int oracle_set_threads(int n);

/* SplitMix64 output function (Steele, Lea & Flood 2014). */
uint64_t oracle_splitmix64(uint64_t x);
/* Tie-break key: sm64(seed ^ sm64((tag << 62) | (L << 32) | j)). */
uint64_t oracle_key(uint64_t seed, uint32_t tag, uint32_t j, uint32_t L);

/* Deb's fast non-dominated sort over all M points, then the front fill:
 * l = min{k : |F_0|+...+|F_k| >= n_stop}. n_stop <= 0 or >= M means N = M.
 * Points in fronts > l get ORACLE_UNRANKED. */
int oracle_nd_sort(const float *F, int M, int m, int n_stop,
                   int *rank, int *front_info);

/* Normalization over S_t = {x : rank[x] <= l}: ideal point, ASF extremes,
 * FP64 intercepts by Gaussian elimination with partial pivoting, fallback to
 * the per-objective maximum when degenerate. Fn rows outside S_t are left
 * untouched. intercept[k] is a_k; extreme[k] the index of extreme point k. */
int oracle_normalize(const float *F, const int *rank, const int *front_info,
                     int M, int m, double *Fn, double *ideal,
                     double *intercept, int *extreme, int *degenerate);

/* Association of every x in S_t with the reference direction of least
 * perpendicular distance (lowest j on ties). Fn is [M][m] FP64, Z is [H][m]
 * float32. Rows outside S_t get pi = -1 and dist = -1. */
int oracle_associate(const double *Fn, const int *rank, const int *front_info,
                     int M, int m, const float *Z, int H, int *pi, double *dist);

/* Niching: the literal one-pick-per-iteration loop of Algorithm 1. */
int oracle_niche(const int *rank, const int *front_info, const int *pi,
                 const double *dist, int M, int H, int N, uint64_t seed,
                 int *selected);

/* The whole selection: nd_sort -> normalize -> associate -> niche.
 * rank_out / pi_out / dist_out may be NULL. */
int oracle_select(const float *F, int M, int m, const float *Z, int H, int N,
                  uint64_t seed, int *selected, int *rank_out, int *pi_out,
                  double *dist_out);

#ifdef __cplusplus
}
#endif
#endif
