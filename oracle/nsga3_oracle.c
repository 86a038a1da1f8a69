/*
 * CPU oracle for NSGA-III environmental selection -- TEST INFRASTRUCTURE.
 *
 * Plain, slow, FP64 code written to be checked against the paper by eye.
 * It is loaded only by the tests, the smoke check and the CPU-baseline leg of
 * the benchmark; the product library never calls it and shares nothing with it.
 *
 * Sources, by function:
 *   dominance / oracle_nd_sort   Sec. II-C (non-dominated sorting of R_t and the
 *                                front fill), Algorithm 1 step "Non-dominated-sort";
 *                                the sort itself is Deb's fast non-dominated sort
 *                                (NSGA-II, cited in the paper's references).
 *   oracle_normalize             Algorithm 1 (associate with normalized objectives),
 *                                Algorithm 2 step "Normalize"; the procedure is
 *                                Deb & Jain 2014 (ideal point, ASF extreme points,
 *                                hyperplane intercepts), which the paper does not
 *                                restate.
 *   oracle_associate             Sec. II-C (association by least perpendicular
 *                                distance to a reference direction), Eq. 1 read as
 *                                the true perpendicular distance ||f|| sin(theta),
 *                                Algorithm 2 (argmin / min over the reference axis).
 *   oracle_niche                 Algorithm 1 (the niche-selection while-loop) and the
 *                                prose that follows it; random choices replaced by
 *                                the SplitMix64 keys below.
 */
#include "nsga3_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- hashing */

/* SplitMix64 output function applied to x (Steele, Lea & Flood, 2014):
 * add the golden gamma, then two xor-shift-multiply rounds and a final
 * xor-shift. All arithmetic is modulo 2^64. */
uint64_t oracle_splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Tie-break key. tag 1 orders reference points at niche level L, tag 2 picks a
 * member of reference j at level L. */
uint64_t oracle_key(uint64_t seed, uint32_t tag, uint32_t j, uint32_t L) {
    uint64_t packed = ((uint64_t)tag << 62) | ((uint64_t)L << 32) | (uint64_t)j;
    return oracle_splitmix64(seed ^ oracle_splitmix64(packed));
}

/* ---------------------------------------------------------------- threads */

/* Threads for the two per-row loops (dominance, association); 1 = the plain
 * serial code. Every result is the same for any count. */
static int g_threads = 1;

int oracle_set_threads(int n) {
    g_threads = n < 1 ? 1 : n;
    return g_threads;
}

/* ----------------------------------------------------- non-dominated sort */

/* a dominates b (minimization): a is no worse in every objective and strictly
 * better in at least one. */
static int dominates(const float *a, const float *b, int m) {
    int strictly_better = 0;
    for (int k = 0; k < m; ++k) {
        double x = a[k], y = b[k];
        if (x > y) return 0;
        if (x < y) strictly_better = 1;
    }
    return strictly_better;
}

static int all_finite(const float *v, long n) {
    for (long i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

typedef struct { int *v; int n, cap; } ivec;

static int ivec_push(ivec *a, int x) {
    if (a->n == a->cap) {
        int cap = a->cap ? 2 * a->cap : 8;
        int *nv = (int *)realloc(a->v, (size_t)cap * sizeof(int));
        if (!nv) return -1;
        a->v = nv;
        a->cap = cap;
    }
    a->v[a->n++] = x;
    return 0;
}

int oracle_nd_sort(const float *F, int M, int m, int n_stop,
                   int *rank, int *front_info) {
    if (!F || !rank || !front_info || M < 1 || m < 1) return -1;
    if (!all_finite(F, (long)M * m)) return -4;
    int N = (n_stop <= 0 || n_stop > M) ? M : n_stop;

    /* S_p: the points p dominates; n_p: how many points dominate p. */
    ivec *S = (ivec *)calloc((size_t)M, sizeof(ivec));
    int *n = (int *)calloc((size_t)M, sizeof(int));
    int *full = (int *)malloc((size_t)M * sizeof(int));
    int *cur = (int *)malloc((size_t)M * sizeof(int));
    int *nxt = (int *)malloc((size_t)M * sizeof(int));
    if (!S || !n || !full || !cur || !nxt) return -5;

    if (g_threads <= 1) {
        for (int p = 0; p < M; ++p) {
            for (int q = p + 1; q < M; ++q) {
                if (dominates(F + (long)p * m, F + (long)q * m, m)) {
                    if (ivec_push(&S[p], q)) return -5;
                    n[q] += 1;
                } else if (dominates(F + (long)q * m, F + (long)p * m, m)) {
                    if (ivec_push(&S[q], p)) return -5;
                    n[p] += 1;
                }
            }
        }
    } else {
        /* Several threads: each row p is built on its own (S_p and n_p from
         * all q), which compares every ordered pair instead of every
         * unordered one but writes no shared state. S_p comes out in the
         * same ascending order as above. */
        int fail = 0;
#pragma omp parallel for schedule(dynamic, 16) num_threads(g_threads) reduction(| : fail)
        for (int p = 0; p < M; ++p) {
            for (int q = 0; q < M; ++q) {
                if (q == p) continue;
                if (dominates(F + (long)p * m, F + (long)q * m, m)) {
                    if (ivec_push(&S[p], q)) fail = 1;
                } else if (dominates(F + (long)q * m, F + (long)p * m, m)) {
                    n[p] += 1;
                }
            }
        }
        if (fail) return -5;
    }

    /* Peel fronts: F_0 = {p : n_p = 0}; removing F_k decrements the counts of
     * everything its members dominate; counts reaching zero form F_{k+1}. */
    int ncur = 0;
    for (int p = 0; p < M; ++p) {
        full[p] = -1;
        if (n[p] == 0) { cur[ncur++] = p; full[p] = 0; }
    }
    int k = 0, cum = 0, l = -1, cum_before_l = 0;
    while (ncur > 0) {
        if (l < 0 && cum + ncur >= N) { l = k; cum_before_l = cum; }
        cum += ncur;
        int nn = 0;
        for (int a = 0; a < ncur; ++a) {
            ivec *sp = &S[cur[a]];
            for (int b = 0; b < sp->n; ++b) {
                int q = sp->v[b];
                if (--n[q] == 0) { full[q] = k + 1; nxt[nn++] = q; }
            }
        }
        int *t = cur; cur = nxt; nxt = t;
        ncur = nn;
        ++k;
    }
    for (int p = 0; p < M; ++p)
        rank[p] = (full[p] <= l) ? full[p] : ORACLE_UNRANKED;
    front_info[0] = l;
    front_info[1] = cum_before_l;
    front_info[2] = N - cum_before_l;
    front_info[3] = l + 1; /* fronts ranked: 0..l (later ones are reported unranked) */

    for (int p = 0; p < M; ++p) free(S[p].v);
    free(S); free(n); free(full); free(cur); free(nxt);
    return (cum == M) ? 0 : -5;
}

/* ----------------------------------------------------------- normalization */

static int in_st(const int *rank, int l, int x) { return rank[x] >= 0 && rank[x] <= l; }

/* Solve E b = 1 by Gaussian elimination with partial pivoting (largest
 * |pivot|, lowest row on ties). Returns 1 if a pivot is below 1e-10 times the
 * largest magnitude of its column in the original matrix. */
static int solve_hyperplane(int m, const double *E, double *b) {
    double *A = (double *)malloc((size_t)m * m * sizeof(double));
    double *r = (double *)malloc((size_t)m * sizeof(double));
    double *colmax = (double *)malloc((size_t)m * sizeof(double));
    int singular = 0;
    if (!A || !r || !colmax) { free(A); free(r); free(colmax); return -1; }
#define A(i, j) A[(size_t)(i) * m + (j)]
    for (int i = 0; i < m; ++i) {
        r[i] = 1.0;
        for (int j = 0; j < m; ++j) A(i, j) = E[i * m + j];
    }
    for (int j = 0; j < m; ++j) {
        colmax[j] = 0.0;
        for (int i = 0; i < m; ++i)
            if (fabs(E[i * m + j]) > colmax[j]) colmax[j] = fabs(E[i * m + j]);
    }
    for (int c = 0; c < m && !singular; ++c) {
        int piv = c;
        for (int i = c + 1; i < m; ++i)
            if (fabs(A(i, c)) > fabs(A(piv, c))) piv = i;
        if (colmax[c] == 0.0 || fabs(A(piv, c)) < 1e-10 * colmax[c]) { singular = 1; break; }
        if (piv != c) {
            for (int j = 0; j < m; ++j) { double t = A(c, j); A(c, j) = A(piv, j); A(piv, j) = t; }
            double t = r[c]; r[c] = r[piv]; r[piv] = t;
        }
        for (int i = c + 1; i < m; ++i) {
            double f = A(i, c) / A(c, c);
            for (int j = c; j < m; ++j) A(i, j) -= f * A(c, j);
            r[i] -= f * r[c];
        }
    }
    for (int i = m - 1; i >= 0 && !singular; --i) {
        double s = r[i];
        for (int j = i + 1; j < m; ++j) s -= A(i, j) * b[j];
        b[i] = s / A(i, i);
    }
#undef A
    free(A); free(r); free(colmax);
    return singular;
}

int oracle_normalize(const float *F, const int *rank, const int *front_info,
                     int M, int m, double *Fn, double *ideal,
                     double *intercept, int *extreme, int *degenerate) {
    if (!F || !rank || !front_info || !Fn || !ideal || !intercept || !extreme ||
        !degenerate || M < 1 || m < 2 || m > ORACLE_MAX_OBJECTIVES)
        return -1;
    int l = front_info[0];
    double *fmax = (double *)malloc((size_t)m * sizeof(double));
    double *E = (double *)malloc((size_t)m * m * sizeof(double));
    double *b = (double *)malloc((size_t)m * sizeof(double));
    if (!fmax || !E || !b) { free(fmax); free(E); free(b); return -5; }

    /* Ideal point z over S_t. */
    for (int k = 0; k < m; ++k) ideal[k] = INFINITY;
    for (int x = 0; x < M; ++x)
        if (in_st(rank, l, x))
            for (int k = 0; k < m; ++k)
                if ((double)F[(long)x * m + k] < ideal[k]) ideal[k] = F[(long)x * m + k];

    /* Largest translated objective over S_t (the fallback intercept). */
    for (int k = 0; k < m; ++k) fmax[k] = 0.0;
    for (int x = 0; x < M; ++x)
        if (in_st(rank, l, x))
            for (int k = 0; k < m; ++k) {
                double v = (double)F[(long)x * m + k] - ideal[k];
                if (v > fmax[k]) fmax[k] = v;
            }

    /* Extreme point for axis k: least ASF with weights 1 on k and 1e-6
     * elsewhere, i.e. max(f'_k, 1e6 * f'_j for j != k); lowest index on ties. */
    for (int k = 0; k < m; ++k) {
        double best = INFINITY;
        int arg = -1;
        for (int x = 0; x < M; ++x) {
            if (!in_st(rank, l, x)) continue;
            double asf = -INFINITY;
            for (int j = 0; j < m; ++j) {
                double fp = (double)F[(long)x * m + j] - ideal[j];
                double v = (j == k) ? fp : 1e6 * fp;
                if (v > asf) asf = v;
            }
            if (asf < best) { best = asf; arg = x; }
        }
        extreme[k] = arg;
    }

    /* Intercepts: the hyperplane sum_j f'_j * b_j = 1 through the m extreme
     * points; a_j = 1 / b_j. */
    for (int k = 0; k < m; ++k)
        for (int j = 0; j < m; ++j)
            E[k * m + j] = (double)F[(long)extreme[k] * m + j] - ideal[j];
    int degen = solve_hyperplane(m, E, b);
    if (degen < 0) { free(fmax); free(E); free(b); return -5; }
    for (int k = 0; k < m && !degen; ++k) {
        if (!(b[k] > 0.0)) { degen = 1; break; }
        double a = 1.0 / b[k];
        if (!isfinite(a) || a < 1e-6 * fmax[k]) { degen = 1; break; }
        intercept[k] = a;
    }
    if (degen) {
        for (int k = 0; k < m; ++k) intercept[k] = (fmax[k] > 0.0) ? fmax[k] : 1.0;
    }
    *degenerate = degen;

    for (int x = 0; x < M; ++x)
        if (in_st(rank, l, x))
            for (int k = 0; k < m; ++k)
                Fn[(long)x * m + k] = ((double)F[(long)x * m + k] - ideal[k]) / intercept[k];
    free(fmax); free(E); free(b);
    return 0;
}

/* ------------------------------------------------------------- association */

int oracle_associate(const double *Fn, const int *rank, const int *front_info,
                     int M, int m, const float *Z, int H, int *pi, double *dist) {
    if (!Fn || !rank || !front_info || !Z || !pi || !dist || M < 1 || m < 1 || H < 1)
        return -1;
    int l = front_info[0];
    double *W = (double *)malloc((size_t)H * m * sizeof(double));
    if (!W) return -5;
    /* Unit reference directions w / ||w||. */
    for (int j = 0; j < H; ++j) {
        double s = 0.0;
        for (int k = 0; k < m; ++k) {
            if (!isfinite(Z[(long)j * m + k]) || Z[(long)j * m + k] < 0.0f) { free(W); return -1; }
            s += (double)Z[(long)j * m + k] * Z[(long)j * m + k];
        }
        if (!(s > 0.0)) { free(W); return -1; }
        s = sqrt(s);
        for (int k = 0; k < m; ++k) W[(long)j * m + k] = Z[(long)j * m + k] / s;
    }
    /* Rows are independent: with several threads each x is still computed
     * by the loop body below, unchanged. */
#pragma omp parallel for schedule(dynamic, 64) num_threads(g_threads > 1 ? g_threads : 1)
    for (int x = 0; x < M; ++x) {
        if (!in_st(rank, l, x)) { pi[x] = -1; dist[x] = -1.0; continue; }
        const double *f = Fn + (long)x * m;
        double best = INFINITY;
        int arg = -1;
        for (int j = 0; j < H; ++j) {
            const double *w = W + (long)j * m;
            /* perpendicular distance: length of f minus its projection on w */
            double p = 0.0;
            for (int k = 0; k < m; ++k) p += f[k] * w[k];
            double s = 0.0;
            for (int k = 0; k < m; ++k) {
                double r = f[k] - p * w[k];
                s += r * r;
            }
            double d = sqrt(s);
            if (d < best) { best = d; arg = j; }
        }
        pi[x] = arg;
        dist[x] = best;
    }
    free(W);
    return 0;
}

/* ------------------------------------------------------------------ niching */

static int cmp_int(const void *a, const void *b) {
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

int oracle_niche(const int *rank, const int *front_info, const int *pi,
                 const double *dist, int M, int H, int N, uint64_t seed,
                 int *selected) {
    if (!rank || !front_info || !pi || !dist || !selected || M < 1 || H < 1 || N < 1 || N > M)
        return -1;
    int l = front_info[0], K = front_info[2];

    int *rho = (int *)calloc((size_t)H, sizeof(int));
    int *cnt = (int *)calloc((size_t)H, sizeof(int));
    int *off = (int *)calloc((size_t)H + 1, sizeof(int));
    int *fill = (int *)calloc((size_t)H, sizeof(int));
    int *mem = (int *)malloc((size_t)M * sizeof(int));
    if (!rho || !cnt || !off || !fill || !mem) return -5;

    /* rho: niche counts of the fully selected fronts S; I_j: members of the
     * last front F_l associated with j, in ascending index order. */
    int nsel = 0;
    for (int x = 0; x < M; ++x) {
        if (rank[x] < 0 || rank[x] > l) continue;
        if (pi[x] < 0 || pi[x] >= H) { nsel = -1; break; }
        if (rank[x] < l) { rho[pi[x]] += 1; selected[nsel++] = x; }
        else cnt[pi[x]] += 1;
    }
    if (nsel < 0) { free(rho); free(cnt); free(off); free(fill); free(mem); return -1; }
    for (int j = 0; j < H; ++j) off[j + 1] = off[j] + cnt[j];
    for (int x = 0; x < M; ++x)
        if (rank[x] == l) mem[off[pi[x]] + fill[pi[x]]++] = x;

    /* One pick per iteration: the least-crowded reference that still has
     * candidates (random among equals -> least tag-1 key), then the nearest
     * member if its niche count is zero, otherwise a random member (tag-2 key
     * modulo the number of remaining members, in ascending index order). */
    for (int picked = 0; picked < K; ++picked) {
        int L = -1;
        for (int j = 0; j < H; ++j)
            if (cnt[j] > 0 && (L < 0 || rho[j] < L)) L = rho[j];
        if (L < 0) break; /* no candidates left: K > |F_l| (bad front_info) */
        int v = -1;
        uint64_t vk = 0;
        for (int j = 0; j < H; ++j) {
            if (cnt[j] == 0 || rho[j] != L) continue;
            uint64_t kj = oracle_key(seed, 1, (uint32_t)j, (uint32_t)L);
            if (v < 0 || kj < vk) { v = j; vk = kj; }
        }
        int *I = mem + off[v];
        int pos;
        if (L == 0) {
            pos = 0;
            for (int a = 1; a < cnt[v]; ++a)
                if (dist[I[a]] < dist[I[pos]]) pos = a; /* ascending order keeps lowest index */
        } else {
            pos = (int)(oracle_key(seed, 2, (uint32_t)v, (uint32_t)L) % (uint64_t)cnt[v]);
        }
        selected[nsel++] = I[pos];
        for (int a = pos; a + 1 < cnt[v]; ++a) I[a] = I[a + 1];
        cnt[v] -= 1;
        rho[v] += 1;
    }
    int ok = (nsel == N);
    qsort(selected, (size_t)nsel, sizeof(int), cmp_int);
    free(rho); free(cnt); free(off); free(fill); free(mem);
    return ok ? 0 : -5;
}

/* ------------------------------------------------------------ whole select */

int oracle_select(const float *F, int M, int m, const float *Z, int H, int N,
                  uint64_t seed, int *selected, int *rank_out, int *pi_out,
                  double *dist_out) {
    if (!F || !Z || !selected || M < 2 || m < 2 || m > ORACLE_MAX_OBJECTIVES || H < 1 || N < 1 ||
        N > M)
        return -1;
    int fi[4];
    int *rank = (int *)malloc((size_t)M * sizeof(int));
    int *pi = (int *)malloc((size_t)M * sizeof(int));
    double *dist = (double *)malloc((size_t)M * sizeof(double));
    double *Fn = (double *)calloc((size_t)M * m, sizeof(double));
    double *ideal = (double *)malloc((size_t)m * sizeof(double));
    double *icpt = (double *)malloc((size_t)m * sizeof(double));
    int *ext = (int *)malloc((size_t)m * sizeof(int));
    int degen;
    int rc = (rank && pi && dist && Fn && ideal && icpt && ext) ? 0 : -5;
    if (!rc) rc = oracle_nd_sort(F, M, m, N, rank, fi);
    if (!rc) rc = oracle_normalize(F, rank, fi, M, m, Fn, ideal, icpt, ext, &degen);
    if (!rc) rc = oracle_associate(Fn, rank, fi, M, m, Z, H, pi, dist);
    if (!rc) rc = oracle_niche(rank, fi, pi, dist, M, H, N, seed, selected);
    if (!rc && rank_out) memcpy(rank_out, rank, (size_t)M * sizeof(int));
    if (!rc && pi_out) memcpy(pi_out, pi, (size_t)M * sizeof(int));
    if (!rc && dist_out) memcpy(dist_out, dist, (size_t)M * sizeof(double));
    free(rank); free(pi); free(dist); free(Fn); free(ideal); free(icpt); free(ext);
    return rc;
}
