/*
 * nsga3.h -- C-ABI of libnsga3.so: NSGA-III environmental selection on an
 * AMD Instinct MI355X (gfx950), one GPU.
 *
 * The calls follow the paper's statement of selection (arXiv 2504.06067):
 * Algorithm 1 (input: merged population R_t = P_t u O_t of size 2N and the
 * reference set Z; output: the next population of size N) and its
 * tensorized restatement Algorithm 2 (normalize, associate, niche counts,
 * niche fill of the last front). nsga3_select runs the four stages in order;
 * the stage calls exist so that each can be driven and checked on its own.
 *
 * Conventions for every call:
 *  - Pointers are DEVICE memory unless marked [host]. The caller owns all
 *    memory; the library never allocates, frees or synchronizes inside a
 *    compute call. Work is enqueued on `stream` (a hipStream_t; NULL means
 *    the null stream) and the call returns at once. Pointers must stay valid
 *    until that work completes.
 *  - Arguments are validated on the host before anything is enqueued. On
 *    NSGA3_EINVAL / NSGA3_EWORKSPACE nothing is enqueued.
 *  - Objectives are minimized. F is row-major [M][m] float32, m in [2, 512]
 *    (kernels specialized per m up to 16; general kernels above, the
 *    many-objective regime of the paper's objective-scaling experiment),
 *    2 <= M <= 2^20. Z is row-major [H][m] float32 with finite, non-negative,
 *    non-zero rows (e.g. a Das-Dennis lattice); the library scales each row
 *    to unit length itself.
 *  - Problems that only the data reveals (non-finite objectives, an invalid
 *    reference row, a broken internal invariant) set a status word inside the
 *    workspace; read it with nsga3_read_status after the work completes.
 *    Outputs are then unspecified (but every write stays in bounds).
 *  - `ws` is a device buffer of at least nsga3_workspace_bytes(M, m, H, N)
 *    bytes, 256-byte aligned. Calls that overlap in time need distinct
 *    workspaces. The status word reflects the most recent call on `ws`.
 *    Nothing in `ws` carries over from one call to the next.
 *  - Ranks are 0-based (the paper's first front F_1 is rank 0). Points in
 *    fronts after the last selected front l are NSGA3_UNRANKED.
 *  - front_info is int32[4] = {l, |S|, K, fronts ranked}: S is the union of
 *    fronts 0..l-1 (all selected) and K = N - |S| >= 1 points are taken from
 *    front l by niching.
 *  - Random tie-breaks (Algorithm 1: the random choice among least-crowded
 *    reference points and of a member) are deterministic functions of `seed`:
 *    key(seed, tag, j, L) = sm64(seed ^ sm64((tag << 62) | (L << 32) | j))
 *    with sm64 the SplitMix64 output function. Among least-crowded
 *    references at niche count L the least tag-1 key goes first; a random
 *    member pick of reference j at niche count L takes the
 *    (key(seed, 2, j, L) mod r)-th of its r remaining candidates in
 *    ascending index order. The result equals the one-pick-per-iteration loop
 *    of Algorithm 1 under these keys, bit for bit.
 */
#ifndef NSGA3_H
#define NSGA3_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    NSGA3_OK = 0,
    NSGA3_EINVAL = -1,      /* bad argument (nothing enqueued) or invalid reference row (status) */
    NSGA3_EWORKSPACE = -2,  /* ws_bytes below nsga3_workspace_bytes (nothing enqueued) */
    NSGA3_EHIP = -3,        /* a HIP runtime call failed */
    NSGA3_ENONFINITE = -4,  /* status: an objective is NaN or infinite */
    NSGA3_EINTERNAL = -5    /* status: an internal invariant failed */
};

#define NSGA3_UNRANKED 0x7fffffff
#define NSGA3_MAX_OBJECTIVES 512
#define NSGA3_MAX_POINTS (1 << 20)

/* Workspace size in bytes for one selection of M merged points, m objectives,
 * H references, N survivors. Pure host function. The dominant term is the
 * bit-packed dominance matrix, ceil(M/64)^2 * 512 bytes. Returns 0 for
 * arguments that every compute call would reject. */
size_t nsga3_workspace_bytes(int32_t M, int32_t m, int32_t H, int32_t N);

/* Non-dominated sorting of the merged population (Sec. II-C; Algorithm 1,
 * "Non-dominated-sort"), then the front fill: l is the first front at which
 * the cumulative size reaches n_stop (n_stop <= 0 or > M means M).
 * Builds the bit-packed dominance matrix (bit i of row j: point i dominates
 * point j), peels fronts with popcounts over it, and stops at front l.
 *   F          [M][m] float32 objectives (read)
 *   rank       int32[M] (write): 0-based front index, NSGA3_UNRANKED after l
 *   front_info int32[4] (write): {l, |S|, K, l + 1}                           */
int nsga3_nd_sort(const float *F, int32_t M, int32_t m, int32_t n_stop,
                  int32_t *rank, int32_t *front_info,
                  void *ws, size_t ws_bytes, void *stream);

/* Normalization of S_t = {x : rank[x] <= l} (Algorithm 1 "associate ...
 * using normalized objectives"; Algorithm 2 "Normalize"), the procedure of
 * Deb & Jain 2014 cited by the paper: ideal point z (least value per
 * objective over S_t); extreme point e_k = argmin over S_t of
 * max(f'_k, 1e6 * max_{j != k} f'_j) with f' = f - z (least index on ties);
 * intercepts a from the hyperplane through the extreme points, solved in
 * FP64 by Gaussian elimination with partial pivoting. If the system is
 * degenerate (pivot below 1e-10 of its column's largest entry, a
 * non-positive or non-finite intercept, or a_k below 1e-6 of the largest f'_k
 * over S_t) every a_k is the largest f'_k over S_t (1 where that is 0).
 * Then Fn = (f - z) / a for rows in S_t.
 *   F, rank, front_info   as produced by nsga3_nd_sort (read)
 *   Fn          [M][m] float32 (write; rows outside S_t untouched)
 *   ideal       float32[m], intercept float64[m], extreme int32[m],
 *   degenerate  int32[1] (0 or 1)                                    (write)  */
int nsga3_normalize(const float *F, const int32_t *rank, const int32_t *front_info,
                    int32_t M, int32_t m, float *Fn, float *ideal, double *intercept,
                    int32_t *extreme, int32_t *degenerate,
                    void *ws, size_t ws_bytes, void *stream);

/* Association (Sec. II-C; Eq. 1 and Algorithm 2, argmin/min over the
 * references): every x in S_t gets the reference j whose direction
 * w_j / ||w_j|| has the least perpendicular distance
 * d = || f - (f . w) w || to Fn[x] (least j on ties).
 *   Fn          [M][m] float32 normalized objectives (read; rows of S_t)
 *   Z           [H][m] float32 reference points (read)
 *   pi          int32[M] (write): reference index; -1 outside S_t
 *   dist        float32[M] (write): perpendicular distance; -1 outside S_t */
int nsga3_associate(const float *Fn, const int32_t *rank, const int32_t *front_info,
                    int32_t M, int32_t m, const float *Z, int32_t H,
                    int32_t *pi, float *dist, void *ws, size_t ws_bytes, void *stream);

/* Niching (Algorithm 1 while-loop; Algorithm 2 nearest and random
 * selection, cache tensor and truncation): niche counts rho over S, then K
 * picks from front l, least-crowded reference first; a reference at niche
 * count 0 takes its nearest candidate (least dist, then least index),
 * otherwise a keyed random one. Output: the N selected indices, ascending.
 *   rank, front_info, pi, dist  (read), selected int32[N] (write)            */
int nsga3_niche(const int32_t *rank, const int32_t *front_info, const int32_t *pi,
                const float *dist, int32_t M, int32_t H, int32_t N, uint64_t seed,
                int32_t *selected, void *ws, size_t ws_bytes, void *stream);

/* The same niche stage as the paper states it (Algorithm 2: nearest
 * selection, then the random selection loop over the cache tensor Q), kept
 * as a baseline to compare with nsga3_niche's closed form on the same GPU.
 * Row j of Q lists the last-front candidates of reference j in the order
 * reference j picks them (nearest first at niche count 0, then the keyed
 * random picks); the loop lets every least-crowded reference take its next
 * row entry per iteration, until K are taken, the last iteration keeping the
 * references with the least tag-1 keys. Same arguments, workspace and
 * result as nsga3_niche (bit for bit). */
int nsga3_niche_cache_tensor(const int32_t *rank, const int32_t *front_info, const int32_t *pi,
                             const float *dist, int32_t M, int32_t H, int32_t N, uint64_t seed,
                             int32_t *selected, void *ws, size_t ws_bytes, void *stream);

/* The whole selection: nd_sort(n_stop = N) -> normalize -> associate ->
 * niche. rank_out int32[M], pi_out int32[M] and dist_out float32[M] may be
 * NULL; when given they receive the intermediate results. */
int nsga3_select(const float *F, int32_t M, int32_t m, const float *Z, int32_t H,
                 int32_t N, uint64_t seed, int32_t *selected, int32_t *rank_out,
                 int32_t *pi_out, float *dist_out,
                 void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------ no alloc
 * For callers that cannot allocate device memory or pass a workspace: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc. nsga3_select with the library's own scratch instead of `ws`:
 * a device array of NSGA3_NOALLOC_SCRATCH_BYTES per GPU, part of the
 * library's code object, held by each GPU the library runs on until the
 * process ends (its address is looked up once per device, at the first call
 * with that device current). The call allocates nothing and enqueues kernels
 * only.
 *  - Arguments as nsga3_select. Returns NSGA3_EINVAL for the same bad
 *    arguments, and NSGA3_EWORKSPACE when nsga3_workspace_bytes(M, m, H, N)
 *    exceeds NSGA3_NOALLOC_SCRATCH_BYTES (e.g. m = 3 holds up to about
 *    M = 22800); nothing is enqueued in either case.
 *  - status: int32[1] device memory or NULL; receives the device-detected
 *    status of the call (the codes of nsga3_read_status) when its work ends.
 *  - Every call on one GPU shares that GPU's scratch, whatever the stream:
 *    calls that overlap in time on one GPU race and give undefined results.
 *    Serialize them (one stream, or events). The scratch keeps the last
 *    call's contents; each call initializes what it needs itself. */
#define NSGA3_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

int nsga3_select_noalloc(const float *F, int32_t M, int32_t m, const float *Z, int32_t H,
                         int32_t N, uint64_t seed, int32_t *selected, int32_t *rank_out,
                         int32_t *pi_out, float *dist_out, int32_t *status, void *stream);

/* ------------------------------------------------------------- batching
 * Many independent selections in one call: every stage runs once over all
 * instances (one grid per kernel, instances of equal m share a launch), so
 * small and uneven instances fill the GPU together. Each instance's result
 * is bit-identical to a plain nsga3_select on the same arguments, whatever
 * the batch around it and whatever its tile parameters.
 *
 * The instance array is [host] memory, read during the call only: the call
 * writes the descriptors into the workspace with its own kernels, so the
 * whole call is a sequence of kernel launches on `stream` (capturable in a
 * HIP graph; a replay reuses the captured descriptors and shapes). */
#define NSGA3_MAX_BATCH 1024

typedef struct nsga3_instance {
    const float *F;       /* [M][m] float32 objectives (read) */
    const float *Z;       /* [H][m] float32 reference points (read) */
    int32_t *selected;    /* int32[N] (write): selected indices, ascending */
    int32_t *rank;        /* int32[M] (write) or NULL: ranks as nsga3_nd_sort */
    int32_t *pi;          /* int32[M] (write) or NULL: reference of each point of S_t */
    float *dist;          /* float32[M] (write) or NULL: its perpendicular distance */
    int32_t M, m, H, N;   /* as nsga3_select */
    uint64_t seed;        /* tie-break seed, as nsga3_select */
    int32_t tile[4];      /* tile parameters, 0 = automatic: [0] 64x64 tiles of the
                           * dominance triangle per work item (1..2^30; automatic:
                           * 1..3, from the tiles of all instances of equal m),
                           * [1] references per
                           * association slice (16..H, a multiple of 16, or H);
                           * [2], [3] must be 0. Results do not depend on them. */
    void *ws;             /* this instance's own workspace region (256-byte aligned,
                           * at least nsga3_instance_workspace_bytes), or NULL: the
                           * region is carved from the call's workspace */
    size_t ws_bytes;      /* size of `ws` */
} nsga3_instance;

/* Workspace bytes of one instance's own region (nsga3_instance.ws); 0 for a
 * shape every call would reject. Pure host function. */
size_t nsga3_instance_workspace_bytes(int32_t M, int32_t m, int32_t H, int32_t N);

/* Workspace bytes of a batched call [host array]: the batch header plus the
 * regions of the instances whose ws is NULL; 0 if any instance or B
 * (1..NSGA3_MAX_BATCH) would be rejected. Pure host function. */
size_t nsga3_batched_workspace_bytes(const nsga3_instance *inst, int32_t B);

/* nsga3_select for every instance of inst[0..B) [host array]. Instances must
 * not share output buffers. Returns NSGA3_EINVAL, with nothing enqueued, for
 * a bad instance, B out of range or a bad tile parameter; NSGA3_EWORKSPACE
 * if ws_bytes is below nsga3_batched_workspace_bytes. */
int nsga3_select_batched(const nsga3_instance *inst, int32_t B, void *ws, size_t ws_bytes,
                         void *stream);

/* Waits for `stream`, then reads the status of every instance of the last
 * batched call on `ws` into status[0..B) [host], each as nsga3_read_status.
 * `inst` and B must be those of that call. (An instance with its own region
 * keeps its status at the start of that region: nsga3_read_status(inst.ws)
 * reads it alone.) */
int nsga3_read_status_batched(const nsga3_instance *inst, int32_t B, const void *ws,
                              void *stream, int32_t *status);

/* ------------------------------------------------------ generation step
 * The step that a served run repeats between selections (Sec. II-C: mating
 * and the variation operators SBX and polynomial mutation produce n
 * offspring; Algorithm 1, "Crossover+Mutation"), for a batch of resident
 * populations, with a synthetic objective map. Not part of the selection.
 * Per slot, decision vectors are row-major float32 [rows][d] in [0, 1),
 * objectives [rows][m]:
 *   NSGA3_EVOLVE_INIT        rows 0..N-1 of X_new/F_new: a uniform random
 *                            population and its objectives (X_old, F_old,
 *                            sel unused)
 *   NSGA3_EVOLVE_POPULATION  rows 0..N-1: the population, row r taken from
 *                            row sel[r] of X_old/F_old (sel NULL: row r)
 *   NSGA3_EVOLVE_GENERATION  the population as above, then N offspring in
 *                            rows N..2N-1: random mating pairs, SBX with
 *                            distribution index 20 on every variable, then
 *                            polynomial mutation (rate 1/d, index 20), values
 *                            clamped to [0, 1 - 2^-24]; F_new = f(X_new)
 * Objective map: y = A (x_1..x_{d-1} - 1/2), u = |y| / ||y||,
 * f = u (1 - 0.3 ln(1 - x_d)). Random draws are SplitMix64 hashes of
 * (seed, generation, individual, variable): a population evolves the same
 * alone or batched. X_new/F_new must not overlap X_old/F_old. */
#define NSGA3_EVOLVE_GENERATION 0
#define NSGA3_EVOLVE_POPULATION 1
#define NSGA3_EVOLVE_INIT 2
#define NSGA3_MAX_EVOLVE_OBJECTIVES 16
#define NSGA3_MAX_DECISION 1024  /* the random draws index variables with 10 bits */

typedef struct nsga3_evolve_slot {
    const float *X_old;   /* [*][d] previous merged decision vectors (read) */
    const int32_t *sel;   /* [N] population rows of X_old/F_old, or NULL (read) */
    const float *F_old;   /* [*][m] their objectives (read) */
    float *X_new;         /* [2N][d] (GENERATION) or [N][d] (write) */
    float *F_new;         /* [2N][m] or [N][m] (write) */
    const float *A;       /* [m][d-1] objective map matrix (read) */
    int32_t N, d, m;      /* N in [1, 2^19], d in [2, NSGA3_MAX_DECISION],
                           * m in [2, NSGA3_MAX_EVOLVE_OBJECTIVES] */
    int32_t generation;   /* in [0, 65535] */
    uint64_t seed;
    int32_t mode;         /* NSGA3_EVOLVE_* */
    int32_t reserved;     /* must be 0 */
} nsga3_evolve_slot;

/* Workspace bytes of a generation step over B slots (descriptor table). */
size_t nsga3_evolve_workspace_bytes(int32_t B);

/* One generation step for slots[0..B) [host array], B in 1..NSGA3_MAX_BATCH.
 * Returns NSGA3_EINVAL (nothing enqueued) for a bad slot. */
int nsga3_evolve_batched(const nsga3_evolve_slot *slots, int32_t B, void *ws, size_t ws_bytes,
                         void *stream);

/* ---------------------------------------------------- quality indicators
 * Measures of what a run produced (not part of the selection), for the
 * paper's quality studies: IGD (Sec. IV, population size against IGD) and
 * the normalized hypervolume of Appendix E. F is a population [n][m]
 * float32, 1 <= n <= 2^20, 2 <= m <= 16.
 *
 * IGD: the mean over the points r of R [nr][m] (points of the optimal
 * front) of min over the population of ||r - f||_2, distances in FP32, the
 * mean in FP64 in a fixed order. *igd (device double) receives it. ws is a
 * device buffer of nsga3_igd_workspace_bytes(nr) bytes, 256-byte aligned. */
size_t nsga3_igd_workspace_bytes(int32_t nr);
int nsga3_igd(const float *F, int32_t n, int32_t m, const float *R, int32_t nr, double *igd,
              void *ws, size_t ws_bytes, void *stream);

/* Hypervolume estimate: *count (device uint64) receives the number of the
 * `samples` sample points of the box [ideal, ref] (ideal, ref: [host] float
 * arrays of m, ideal_k <= ref_k) that some population point weakly dominates
 * (f_k <= y_k for every k). The normalized hypervolume HV / HV_max of the
 * paper is count / samples, with ideal = 0.9 f_min and ref = 1.01 f_max.
 * Sample i, objective k: u = (sm64(seed ^ sm64(i << 8 | k)) >> 40) * 2^-24
 * and y_k = ideal_k + u * (ref_k - ideal_k), each FP32 operation rounded
 * separately (no fused multiply-add). samples in [1, 2^31]. */
int nsga3_hv_count(const float *F, int32_t n, int32_t m, const float *ideal, const float *ref,
                   int64_t samples, uint64_t seed, unsigned long long *count, void *stream);

/* Waits for `stream`, then reads the status word of `ws` into *status [host]
 * (NSGA3_OK, NSGA3_ENONFINITE, NSGA3_EINVAL or NSGA3_EINTERNAL). Returns
 * NSGA3_OK, or NSGA3_EHIP if the copy or the wait failed. */
int nsga3_read_status(const void *ws, void *stream, int32_t *status);

/* Library version string [host, static storage]. */
const char *nsga3_version(void);

/* Instrumentation (host, not thread-safe). nsga3_profile_enable(names)
 * starts recording a pair of HIP events around every later launch of the
 * named kernels, on the stream of the call that launches them: `names` is a
 * comma-separated list of kernel names ("dominance", "peel", "associate",
 * ...), "*" for all, NULL or "" to stop. It creates its event pool up front
 * (no allocation happens at launch time), clears earlier records and returns
 * NSGA3_OK, NSGA3_EINVAL (list too long) or NSGA3_EHIP. Up to 8192 launches
 * are recorded; later ones are counted as dropped.
 * nsga3_profile_read waits for the recorded events of `kernel` and returns
 * the summed milliseconds and the number of launches (and the dropped count). */
int nsga3_profile_enable(const char *names);
int nsga3_profile_read(const char *kernel, double *total_ms, int64_t *launches,
                       int32_t *dropped);

#ifdef __cplusplus
}
#endif
#endif /* NSGA3_H */
