/*
 * prot — push-relabel additive epsilon-approximation of the assignment
 * problem on one AMD Instinct MI355X (gfx950).
 *
 * Method: Lahn, Raghvendra and Zhang, "A Push-Relabel Based Additive
 * Approximation for Optimal Transport" (arXiv:2203.03732), Section 2.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Supply vertices B are matrix ROWS (points X), demand vertices A are
 *    matrix COLUMNS (points Y). n = |A| = |B| (balanced case, Section 2).
 *  - Rounded costs are int16 units of eps: cbar(a,b) = eps * k[b][a]
 *    (Section 2.1, eq. (1)). Dual weights are int32 units of eps
 *    (the duals stay integer multiples of eps, Section 2.2).
 *  - Every array argument is a DEVICE pointer owned by the caller; the
 *    library never frees or retains it past the call. Only `prot_stats*`
 *    arguments and the `*_host` arrays are host pointers.
 *  - Work is enqueued on the context's HIP stream. A call that fills a
 *    host `prot_stats` synchronises that stream before returning.
 *  - Every function returns PROT_OK (0), PROT_PARTIAL (1) or a negative
 *    error code. No C++ exception crosses this boundary.
 *    prot_last_error(ctx) returns a message for the last failing call.
 *  - A context is not thread-safe: use one per host thread / stream.
 *  - The matrix layout is row-major with a row pitch (in elements) of
 *    prot_pitch(n): n rounded up to a multiple of 128 (256-byte rows).
 */
#ifndef PROT_H
#define PROT_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct prot_ctx prot_ctx;

enum {
    PROT_OK = 0,
    PROT_PARTIAL = 1,          /* stopped at opts->max_phases; state valid */
    PROT_E_ARG = -1,           /* null pointer, bad size or bad option */
    PROT_E_RANGE = -2,         /* a cost is NaN or outside [0, 1] */
    PROT_E_EPS = -3,           /* eps not in (0,1), or 1/eps too big for int16 */
    PROT_E_PHASE_BOUND = -4,   /* the phase-bound watchdog stopped the loop; state valid */
    PROT_E_STATE = -5,         /* warm-start state violates (I1)/(I2) or is not a matching */
    PROT_E_HIP = -6,           /* a HIP runtime call failed */
    PROT_E_NOMEM = -7,         /* device allocation failed */
    PROT_E_UNSUPPORTED = -8    /* size beyond the library's limits */
};

enum { PROT_EPS_ALGORITHMIC = 0, PROT_EPS_STRICT = 1 };
enum { PROT_COST_DIRECT = 0, PROT_COST_MATRIX_CORES = 1, PROT_COST_AUTO = 2 };
enum { PROT_COSTS_AUTO = 0, PROT_COSTS_MATRIX = 1, PROT_COSTS_ON_THE_FLY = 2 };
enum { PROT_ORIGIN_DIAG = 0, PROT_ORIGIN_ZERO = 1 };
enum { PROT_KTYPE_AUTO = 0, PROT_KTYPE_INT16 = 1, PROT_KTYPE_UINT8 = 2 };
enum { PROT_METRIC_SQEUCLIDEAN = 0, PROT_METRIC_EUCLIDEAN = 1, PROT_METRIC_L1_NORMALIZED = 2 };

typedef struct {
    /* PROT_EPS_ALGORITHMIC runs with the given eps (additive error 3 eps n,
     * Section 2.1); PROT_EPS_STRICT runs with eps/3 (error eps n). */
    int32_t eps_mode;
    /* Scan order of the greedy step: row b starts at column b and wraps
     * (PROT_ORIGIN_DIAG, default) or starts at column 0 (PROT_ORIGIN_ZERO). */
    int32_t origin_mode;
    /* 1: skip the arbitrary completion (Section 2.1), return the phase-loop
     * matching as is. */
    int32_t no_completion;
    /* Point-set solves: where the rounded costs live. PROT_COSTS_MATRIX
     * builds the n x n int16 matrix and scans it; PROT_COSTS_ON_THE_FLY
     * (d = 2, 3) builds only the maximum and the threshold table and lets
     * the greedy step recompute each k it examines from the points with the
     * build's own operations (identical integers, no n^2 memory);
     * PROT_COSTS_AUTO stores a matrix of up to 256 MiB and otherwise
     * recomputes, and a solve that returns statistics then hands over to the
     * stored matrix (up to 16 GiB, if it can be allocated) once the loop has
     * run about twice as long as writing the matrix would take: the loop
     * stops at a phase start and resumes on the matrix from the state
     * reached, with the same results (two loop launches). */
    int32_t cost_storage;
    /* Element type of the rounded-cost matrix that solve_cost / solve_points
     * store: PROT_KTYPE_AUTO (= int16), PROT_KTYPE_INT16, PROT_KTYPE_UINT8
     * (K = floor(1/eps_internal) <= 253, else PROT_E_UNSUPPORTED). Bytes halve
     * the matrix's memory and the cost build's writes (a larger instance fits
     * HBM or the Infinity Cache); the scan reads half the bytes but widens
     * them to int16 lanes and is not faster on MI355X. The costs and every
     * result are the same. */
    int32_t k_type;
    /* Warm starts of prot_solve_rounded*: 1 also checks (I2) on every edge,
     * y(a) + y(b) <= k + 1 and = k on the matching (eqs. (2), (3); O(n_b n_a)
     * reads of k), before the loop; a violation returns PROT_E_STATE. The
     * O(n) checks always run: a matching, (I1), and |y| <= K + 2 (Lemma 3.2,
     * K = 32765 for prot_solve_rounded*, floor(1/eps) otherwise). */
    int32_t check_warm;
    /* The watchdog. 0 (default): the loop may run at most
     * ((n_b + n_a)(K + 2) - n_b) / (T + 1) phases, the bound that Lemma 3.2
     * (|y| <= K + 2) and Lemma 3.3 (each phase adds |B'| > T to
     * sum y(b) - sum y(a)) give every run of the method; eq. (4)'s printed
     * constant counts the 2n duals once, this bound counts them as Lemma 3.2
     * does. Reaching it returns PROT_E_PHASE_BOUND with the state reached in
     * the outputs (no completion), which a warm start can resume. > 0: that
     * many phases instead; < 0: no watchdog. */
    int64_t phase_bound;
    /* Stop after this many phases (0: run to completion); the call then
     * returns PROT_PARTIAL and the outputs hold a valid resumable state. */
    int64_t max_phases;
} prot_opts;

typedef struct {
    int64_t phases;            /* phases run (Section 2.2) */
    int64_t sum_free;          /* sum over phases of |B'| */
    int64_t rounds;            /* proposal rounds that made a proposal */
    int64_t max_rounds;        /* most such rounds in one phase */
    int64_t scanned;           /* matrix entries examined by the greedy step */
    int64_t matched_in_phases; /* |M| when the phase loop stopped */
    int64_t completed_pairs;   /* pairs added by the completion */
    int64_t sum_k;             /* sum of k over the returned matching */
    int64_t threshold;         /* T: the loop stops when |B'| <= T */
    int32_t kmax;              /* largest rounded cost */
    int32_t status;            /* PROT_OK, PROT_PARTIAL or PROT_E_PHASE_BOUND */
    double cost;               /* sum of c(a,b) over the matching (costs scaled to max 1) */
    double cost_scale;         /* points: the maximum squared distance m (c = d2/m); cost input: 1 */
    double eps_internal;       /* eps the loop ran with (eps or eps/3) */
    double ms_build;           /* device time of the cost build (0 if none) */
    double ms_loop_kernel;     /* device time of the persistent phase-loop kernel */
    double ms_total;           /* device time from the first kernel to the last */
} prot_stats;

/* Create a context on `device` that enqueues on `hip_stream` (a hipStream_t
 * passed as void*, NULL = the null stream). */
int prot_ctx_create(prot_ctx **out, int device, void *hip_stream);
int prot_ctx_destroy(prot_ctx *ctx);
/* Change the stream later calls enqueue on. */
int prot_set_stream(prot_ctx *ctx, void *hip_stream);

/* How later point-set cost builds on ctx (and batches created afterwards)
 * compute the squared distances; all give the same result, bit for bit.
 * PROT_COST_DIRECT: every distance as the fma-accumulated sum of squared
 * coordinate differences, the definition itself (Section 2.1 rounds these
 * costs by eq. (1)); two vector instructions per coordinate and pair.
 * PROT_COST_MATRIX_CORES: for d >= 16, |x|^2 + |y|^2 - 2 x.y with FP32
 * matrix-core products (one multiply-add per coordinate and pair, at twice
 * the FP32 rate of the unpacked vector units this library uses) plus a
 * rounding-error bound; entries the bound cannot place in their rounding
 * cell, and the pairs that may hold the maximum, are recomputed directly.
 * PROT_COST_AUTO (default): the matrix cores from d = 48 on, where they
 * measured faster on MI355X, the direct path below. The matrix cores serve
 * the squared cost of balanced instances and batches; other builds take the
 * direct path. Returns PROT_E_ARG for an unknown path. */
int prot_set_cost_path(prot_ctx *ctx, int32_t path);
/* The cost of a pair in later single-instance point-set builds and solves on
 * ctx (prot_build_costs*, prot_solve_points*; batches always use the squared
 * cost). All are scaled to at most 1 and rounded by eq. (1) in binary64.
 * PROT_METRIC_SQEUCLIDEAN (default): d2 / m, d2 the fma-accumulated binary32
 * squared distance, m its maximum over all pairs. PROT_METRIC_EUCLIDEAN
 * (Section 5's synthetic experiment): sqrt(d2 / m) in binary64; every entry
 * is placed exactly through a table of the smallest binary32 d2 reaching
 * each k. PROT_METRIC_L1_NORMALIZED (Section 5's image experiment): every
 * vector is divided by its sum (binary32, sum in coordinate order), the cost
 * is half the L1 distance of the normalised vectors (binary32, coordinate
 * order) clamped to 1; entries must be finite and nonnegative with a
 * positive sum (PROT_E_RANGE otherwise), d <= 12288; m_out and cost_scale
 * report 2. The last two store the matrix (PROT_COSTS_ON_THE_FLY returns
 * PROT_E_UNSUPPORTED; AUTO stores it). Returns PROT_E_ARG for an unknown
 * metric. */
int prot_set_cost_metric(prot_ctx *ctx, int32_t metric);
/* Pre-size the workspace for instances up to n_max (and, if with_matrix,
 * an n_max x prot_pitch(n_max) int16 cost matrix) so that later calls do
 * not allocate. */
int prot_reserve(prot_ctx *ctx, int64_t n_max, int32_t with_matrix);

/* Row pitch in elements used for int16 rounded-cost matrices. */
int64_t prot_pitch(int64_t n);
/* Integer stop threshold T = floor(eps * n + 1e-9) (Section 2.2:
 * stop once |B'| <= eps n). */
int64_t prot_threshold(double eps, int64_t n);
/* Largest n the single-instance phase loop accepts on this device. */
int64_t prot_max_n(prot_ctx *ctx);

/* eq. (1): k[b*ldk + a] = floor(C[b*ldc + a] / eps), the division in
 * binary64. C: n x n float32 scaled to [0, 1]. Returns PROT_E_RANGE if
 * any cost is NaN or outside [0, 1] (k is then unspecified). ldk >= n. */
int prot_round_costs(prot_ctx *ctx, const float *C, int64_t n, int64_t ldc,
                     double eps, int16_t *k, int64_t ldk);

/* Rounded squared-Euclidean costs from point sets (Section 1 scaling, eq. (1)):
 * X: n x d (rows B), Y: n x d (columns A), float32 row-major.
 * d2 = sum_j fma-accumulated (x_j - y_j)^2 in binary32 in coordinate order,
 * m = max d2, k = floor((d2 / m) / eps) with both divisions in binary64
 * (k = 0 everywhere if m = 0). k: n x ldk int16 (columns ldk > n are filled
 * with 0x7FFF). m is written to *m_out (device float) if non-null. */
int prot_build_costs(prot_ctx *ctx, const float *X, const float *Y, int64_t n,
                     int32_t d, double eps, int16_t *k, int64_t ldk,
                     float *m_out);

/* The integer phase loop of Section 2.2 on rounded costs k (n x ldk int16,
 * 0 <= k <= 32765), stopping once |B'| <= T, then the completion.
 *  warm = 0: start from y(b) = 1, y(a) = 0, M empty (mate_* and y_* are
 *            outputs only).
 *  warm = 1: resume from the state in mate_a, mate_b, y_a, y_b (it must be
 *            a matching satisfying (I1) with |y| <= 32767, and (I2) when
 *            opts->check_warm is set; PROT_E_STATE otherwise).
 * Outputs: mate_a[a] (b or -1), mate_b[b] (a or -1), and the duals y_a, y_b
 * BEFORE the completion (completion edges carry no eq. (3) guarantee).
 * stats may be NULL: then the call only enqueues (no synchronisation) and
 * prot_ctx_status reports how the work ended. If the loop fails on the
 * device (a bounded wait timed out, a dual left its range), the completion
 * is skipped and every mate is -1. With stats, a loop that could not start
 * because too few workgroups were resident at once (another kernel holds
 * the GPU) is run again with a cooperative launch, which waits for them. */
int prot_solve_rounded(prot_ctx *ctx, const int16_t *k, int64_t n, int64_t ldk,
                       int64_t T, const prot_opts *opts, int32_t warm,
                       int32_t *mate_a, int32_t *mate_b, int32_t *y_a,
                       int32_t *y_b, prot_stats *stats);

/* Cost-matrix input: prot_round_costs into workspace, then the phase loop
 * with T = prot_threshold(eps_internal, n), then the completion; stats->cost
 * is sum_b C[b][mate_b[b]] in binary64. */
int prot_solve_cost(prot_ctx *ctx, const float *C, int64_t n, int64_t ldc,
                    double eps, const prot_opts *opts, int32_t *mate_a,
                    int32_t *mate_b, int32_t *y_a, int32_t *y_b,
                    prot_stats *stats);

/* Point-set input: prot_build_costs into workspace, then as above;
 * stats->cost is sum_b d2_64(b, mate_b[b]) / m in binary64 (normalised),
 * stats->cost_scale = m. stats = NULL enqueues only (no synchronisation,
 * no cooperative retry); prot_ctx_status then reports how the solve ended. */
int prot_solve_points(prot_ctx *ctx, const float *X, const float *Y,
                      int64_t n, int32_t d, double eps, const prot_opts *opts,
                      int32_t *mate_a, int32_t *mate_b, int32_t *y_a,
                      int32_t *y_b, prot_stats *stats);

/* The unbalanced case (Section 3.3, Lemma 3.5): |B| = n_b rows (supply)
 * and |A| = n_a >= n_b columns (demand). The algorithm is unchanged; the
 * loop stops when |B'| <= T = floor(eps_internal n_b), giving a matching of at
 * least (1 - eps)|B| rows whose rounded cost is within eps |B| of an optimal
 * |B|-matching; the completion then gives every row a column (the i-th free
 * b takes the i-th free a). Layouts as for the square calls, with n_b rows of
 * n_a columns: k and C are n_b x ld (ld >= n_a), X is n_b x d, Y is n_a x d;
 * mate_b and y_b have n_b entries, mate_a and y_a n_a (mate_a = -1 for the
 * n_a - n_b columns left unmatched). n_a < n_b returns PROT_E_ARG (transpose
 * the input). n_b = 0 with n_a > 0 writes the cold-start column state
 * (mate_a = -1, y_a = 0; untouched when warm). The square calls are these
 * with n_b = n_a = n. Sizes of the phase loop (every solve call): each
 * workgroup keeps the duals of all n_a columns in its LDS up to about 81,000
 * columns on MI355X, and in global memory beyond (2 * n_a bytes per
 * workgroup of the loop, allocated by the context); a row index travels in 17
 * bits up to n_b = 131,071 and in 18 bits up to 262,143, where the row duals
 * must stay below 16,384 (eps >= 1/16381 for point sets; a given matrix
 * whose duals outgrow that stops with PROT_E_STATE). Larger n_b returns
 * PROT_E_UNSUPPORTED. */
int prot_round_costs_rect(prot_ctx *ctx, const float *C, int64_t n_b, int64_t n_a,
                          int64_t ldc, double eps, int16_t *k, int64_t ldk);
int prot_build_costs_rect(prot_ctx *ctx, const float *X, int64_t n_b, const float *Y,
                          int64_t n_a, int32_t d, double eps, int16_t *k, int64_t ldk,
                          float *m_out);
int prot_solve_rounded_rect(prot_ctx *ctx, const int16_t *k, int64_t n_b, int64_t n_a,
                            int64_t ldk, int64_t T, const prot_opts *opts, int32_t warm,
                            int32_t *mate_a, int32_t *mate_b, int32_t *y_a,
                            int32_t *y_b, prot_stats *stats);
int prot_solve_cost_rect(prot_ctx *ctx, const float *C, int64_t n_b, int64_t n_a,
                         int64_t ldc, double eps, const prot_opts *opts, int32_t *mate_a,
                         int32_t *mate_b, int32_t *y_a, int32_t *y_b, prot_stats *stats);
int prot_solve_points_rect(prot_ctx *ctx, const float *X, int64_t n_b, const float *Y,
                           int64_t n_a, int32_t d, double eps, const prot_opts *opts,
                           int32_t *mate_a, int32_t *mate_b, int32_t *y_a,
                           int32_t *y_b, prot_stats *stats);

/* ---- Batches of independent instances (minibatch optimal transport) ---- */

/* Per-instance results of a batched solve. */
typedef struct {
    int64_t phases, sum_free, rounds, max_rounds, scanned, matched_in_phases,
        completed_pairs, sum_k, threshold;
    int32_t status;            /* PROT_OK, PROT_PARTIAL or PROT_E_PHASE_BOUND */
    int32_t kmax;
    double cost;               /* sum over the matching of d2 / m, binary64 */
    double cost_scale;         /* m, the instance's max squared distance */
} prot_instance_stats;

/* Optimal transport (Section 4). The supplies nu (n_b points, the rows of
 * C) and demands mu (n_a points, the columns) are probability vectors;
 * C (row-major, ldc >= n_a) holds costs in [0, 1].
 *   1. Scaling: theta = 4 max(n_b, n_a) / eps_internal; supply point b
 *      becomes floor(theta nu_b) unit copies, demand point a
 *      ceil(theta mu_a) (binary64 products); copies of a point are
 *      contiguous, in point order.
 *   2. The phase loop of Section 2.2 on the unbalanced instance of copies
 *      (rows: supply copies, columns: demand copies; a copy's rounded cost is
 *      eq. (1) of its points' cost), stopping at |B'| <= floor(eps_internal x
 *      supply copies), with the invariant of Section 4: after every phase
 *      each free supply copy's dual is raised to the largest dual among the
 *      copies of its point. The completion then matches every supply copy.
 *   3. The plan: 1/theta per matched pair of copies, made feasible by a
 *      repair the paper leaves implicit: a demand point holding more than
 *      mu_a (its copies were rounded up) returns the excess, taken from its
 *      edges in ascending b; the mass still to be sent is then paired with
 *      the room left at the demand points in index order (north-west corner
 *      rule on the running totals). The result sends exactly nu_b from each
 *      b (to rounding) and at most mu_a into each a; its cost is within
 *      3 eps + eps/2 of the optimal transport cost (ALGORITHMIC eps).
 * Outputs (device memory owned by the caller): plan, n_b x ldp binary64
 * (written only when the call returns PROT_OK); the duals in the
 * two-cluster form of Lemma 4.1: for each point the smaller dual of its
 * copies (units of eps_internal) and how many copies hold it, the others
 * holding that value + 1 (points without copies: 0 and 0). Errors:
 * PROT_E_RANGE for masses that are not probability vectors or costs outside
 * [0, 1]; PROT_E_UNSUPPORTED when the demand copies exceed the column-dual
 * capacity of one workgroup's LDS (about 81,000: theta + n_a must fit).
 * opts: eps_mode, origin_mode and max_phases apply (no_completion is
 * ignored); with PROT_PARTIAL the plan is not valid. */
typedef struct {
    double theta;              /* 4 max(n_b, n_a) / eps_internal */
    int64_t copies_b;          /* sum floor(theta nu_b) */
    int64_t copies_a;          /* sum ceil(theta mu_a) */
    double repaired_mass;      /* mass moved by the feasibility repair (<= eps/2) */
    prot_stats loop;           /* the phase loop on the copies; loop.cost is the plan's cost */
} prot_ot_stats;

int prot_ot_solve(prot_ctx *ctx, const float *C, int64_t n_b, int64_t n_a, int64_t ldc,
                  const double *nu, const double *mu, double eps, const prot_opts *opts,
                  double *plan, int64_t ldp, int32_t *y_b_lo, int32_t *y_b_nlo,
                  int32_t *y_a_lo, int32_t *y_a_nlo, prot_ot_stats *stats);

/* Optimal transport (Section 4) with the copies of every point kept as two
 * dual clusters (Lemma 4.1), so that the state is O(n_b + n_a) per side
 * plus the pair counts, whatever theta. Same problem, arguments, outputs and
 * errors as prot_ot_solve, and the same scaling, rounding, stop threshold,
 * completion reading, plan and repair; the phases are taken point by point:
 *   - supply point b keeps Y_b (the larger dual of its copies; its free
 *     copies sit there after the free-copy raise) and its free count; demand
 *     point a keeps Z_a (the larger dual of its copies) and its free count;
 *     a matched pair of copies is tight (eq. (2)), so the pairs between b
 *     and a are counted by the parity of the demand copy's level;
 *   - step (I): edge (a, b) is admissible for b's free copies exactly when
 *     k + 1 = Z_a + Y_b (the lower level of a never is, by (I1)). In
 *     synchronous rounds every b with copies still looking asks the first
 *     admissible point in its scan order (DIAG: from column b mod n_a) that
 *     had top-level copies left when the round began for all of them; a
 *     point serves its proposers in ascending b as far as its top copies
 *     go; a b served in part or not at all goes on after that point;
 *   - step (II): a point hands out the copies taken from its free ones
 *     first, then from those matched at Z_a in ascending order of the
 *     partner point, whose copies become free;
 *   - step (III): the taken copies drop one step (Z_a drops when all top
 *     copies went); a b with copies left over rises one step; freed copies
 *     take the largest dual of their point.
 * This is one admissible run of the copies' algorithm (a maximal M' in
 * every phase), so the guarantees of prot_ot_solve hold; the matching it
 * picks differs from prot_ot_solve's copy-by-copy rounds. Limits: at most
 * 4096 points a side (the points' state is held by one workgroup);
 * sum ceil(theta mu_a) < 2^31. loop.scanned counts the positions the
 * point-level scans pass, as in a scan of the n_a columns of each point. */
int prot_ot_solve_clustered(prot_ctx *ctx, const float *C, int64_t n_b, int64_t n_a,
                            int64_t ldc, const double *nu, const double *mu, double eps,
                            const prot_opts *opts, double *plan, int64_t ldp, int32_t *y_b_lo,
                            int32_t *y_b_nlo, int32_t *y_a_lo, int32_t *y_a_nlo,
                            prot_ot_stats *stats);

typedef struct prot_batch prot_batch;

/* Largest n of one instance in a batch. */
int32_t prot_batch_max_n(void);

/* Plan a batch of `batch` independent point-set instances (squared Euclidean
 * cost scaled per instance to max 1, eq. (1) rounding, the phase loop of
 * Section 2.2, the completion). Instance i has n_host[i] points
 * (1 <= n_host[i] <= prot_batch_max_n()) stored in rows [o_i, o_i + n_host[i])
 * of X and Y (float32, d columns) and of every output array, with
 * o_i = n_host[0] + ... + n_host[i-1]; output mates are indices local to the
 * instance. n_host is a host array read during the call. The plan owns its
 * device workspace (metadata, one rounded-cost matrix per instance). */
int prot_batch_create(prot_ctx *ctx, int32_t batch, const int64_t *n_host, int32_t d,
                      double eps, const prot_opts *opts, prot_batch **out);

/* How a batch runs (results are the same for every choice):
 *   engine   PROT_BATCH_ENGINE_LDS: one workgroup solves a whole instance
 *            with its state in LDS (n <= 2048); PROT_BATCH_ENGINE_TEAMS:
 *            `team` workgroups of the persistent phase loop per instance;
 *            PROT_BATCH_ENGINE_AUTO: LDS up to n_max = 1024, teams above.
 *   team     TEAMS: workgroups per instance, 1..8 (0: as many as fit);
 *            PROT_E_UNSUPPORTED if fewer than ceil(n_max / 1024) or more
 *            than fit next to each other on the GPU.
 *   cost_path  PROT_COST_DIRECT / PROT_COST_MATRIX_CORES / PROT_COST_AUTO, or
 *            -1 for the context's setting. */
enum { PROT_BATCH_ENGINE_AUTO = 0, PROT_BATCH_ENGINE_LDS = 1, PROT_BATCH_ENGINE_TEAMS = 2 };
typedef struct {
    int32_t engine;
    int32_t team;
    int32_t cost_path;
    int32_t reserved;
} prot_batch_config;

/* prot_batch_create with an explicit configuration (NULL = automatic). */
int prot_batch_create_config(prot_ctx *ctx, int32_t batch, const int64_t *n_host, int32_t d,
                             double eps, const prot_opts *opts, const prot_batch_config *cfg,
                             prot_batch **out);

/* Autotuner: times every configuration that applies to this batch (the LDS
 * engine, teams of each size that fits, both cost paths for d >= 16) on
 * the caller's inputs X, Y (device, the plan's packed layout), each run
 * once to warm up and then `reps` times (HIP events on the context
 * stream), and returns the fastest in *best, its mean time in *best_ms and
 * the number of configurations timed in *tried. Allocates its own
 * scratch outputs; synchronises the stream. */
int prot_batch_autotune(prot_ctx *ctx, int32_t batch, const int64_t *n_host, int32_t d,
                        double eps, const prot_opts *opts, const float *X, const float *Y,
                        int32_t reps, prot_batch_config *best, double *best_ms,
                        int32_t *tried);
int prot_batch_destroy(prot_batch *plan);

/* Enqueue the whole batched solve on the context stream; no synchronisation
 * (prot_batch_status reports how it ended). stats: device array of `batch`
 * entries, or NULL. An instance's loop stops at the phase bound of
 * prot_opts.phase_bound (status PROT_E_PHASE_BOUND in its statistics). */
int prot_batch_run(prot_batch *plan, const float *X, const float *Y, int32_t *mate_a,
                   int32_t *mate_b, int32_t *y_a, int32_t *y_b, prot_instance_stats *stats);

/* Capture the work of prot_batch_run with these pointers into a HIP graph
 * (replacing any earlier capture of this plan), and replay it on the
 * context stream. The pointers must stay valid while the graph is used. */
int prot_batch_capture(prot_batch *plan, const float *X, const float *Y, int32_t *mate_a,
                       int32_t *mate_b, int32_t *y_a, int32_t *y_b, prot_instance_stats *stats);
int prot_batch_replay(prot_batch *plan);

/* Convenience: plan, run, synchronise, copy the per-instance statistics to
 * stats_host (host array of `batch` entries, may be NULL), free the plan.
 * Returns PROT_E_RANGE if a coordinate is not finite. */
int prot_solve_batched_points(prot_ctx *ctx, int32_t batch, const int64_t *n_host, int32_t d,
                              const float *X, const float *Y, double eps,
                              const prot_opts *opts, int32_t *mate_a, int32_t *mate_b,
                              int32_t *y_a, int32_t *y_b, prot_instance_stats *stats_host);

/* Matching-based OT loss of every instance of a plan, from its matching:
 * L_i = (1/n_i) * sum_b ||x_b - y_{mate_b[b]}||^2 (float32 result of a
 * binary64 sum; unmatched rows add nothing). X, Y and mate_b use the plan's
 * packed layout; loss: device float[batch]. */
int prot_batch_loss_fwd(prot_batch *plan, const float *X, const float *Y,
                        const int32_t *mate_b, float *loss);

/* Gradient of sum_i g_i * L_i for the fixed matching (the matching is
 * piecewise constant in X and Y): dX_b = (2 g_i / n_i)(x_b - y_{mate_b[b]}),
 * dY_a = (2 g_i / n_i)(y_a - x_{mate_a[a]}), 0 where unmatched. grad_loss:
 * device float[batch]; dX, dY: device, same layout as X, Y. */
int prot_batch_loss_bwd(prot_batch *plan, const float *X, const float *Y,
                        const int32_t *mate_a, const int32_t *mate_b,
                        const float *grad_loss, float *dX, float *dY);

/* Per-phase record of the last phase loop on this context: for phase i,
 * out[4i..4i+3] = (|B'|, rounds, scanned entries, |M'|). Copies at most cap
 * phases and returns the number of phases recorded (<= the trace capacity,
 * 65536). Synchronises the stream. */
int64_t prot_get_trace(prot_ctx *ctx, int64_t *out_host, int64_t cap);

/* Diagnostics: per-round device timestamps of the last phase loop, recorded
 * only when the context was created with PROT_DEBUG_ROUND_TIMES=1 in the
 * environment. For round r (0-based), out[3r] = latest arrival of any
 * workgroup at the round's grid barrier, out[3r+1] = the barrier's exit,
 * out[3r+2] = the phase index; times in ticks of the 100 MHz device clock,
 * 0 for rounds not run. Returns the number of rounds copied (0 if timing is
 * off). Synchronises the stream. */
int64_t prot_get_round_times(prot_ctx *ctx, int64_t *out_host, int64_t cap);

/* Device times (ms) of the last `count` phase-loop launches on ctx, oldest
 * first, from events that the launches themselves carry (each solve, warm
 * start or transport call launches the loop once; the context keeps the
 * last 1,024). For timing solves enqueued with stats = NULL, which report no
 * statistics. ms_out: host array of at least `count` floats. Synchronises the
 * stream; returns the number of times written (<= count), or
 * PROT_E_ARG / PROT_E_HIP. */
int32_t prot_loop_times(prot_ctx *ctx, float *ms_out, int32_t count);

/* How the work last enqueued on ctx by a solve call ended: synchronises
 * the context stream and returns PROT_OK, PROT_PARTIAL, PROT_E_PHASE_BOUND
 * or the error the device reported (PROT_E_RANGE for a non-finite or
 * out-of-range input, PROT_E_STATE, PROT_E_HIP for a timed-out wait or too
 * few resident workgroups, PROT_E_UNSUPPORTED). For calls made with
 * stats = NULL, which do not synchronise. */
int prot_ctx_status(prot_ctx *ctx);

/* How the last run or replay of a batch plan ended (synchronises the
 * context stream): PROT_OK, PROT_E_RANGE (a coordinate is not finite),
 * PROT_E_PHASE_BOUND (an instance was stopped by the watchdog, its
 * statistics say which), PROT_E_HIP / PROT_E_STATE / PROT_E_UNSUPPORTED (an
 * instance's loop failed). */
int prot_batch_status(prot_batch *plan);

/* The matching-based OT loss without a batch plan: `batch` instances of n
 * points each, X and Y batch x n x d float32 (row-major, instance after
 * instance), mate_b batch x n int32 (row b of an instance -> its column,
 * local to the instance; -1 = unmatched, adds nothing), all device memory:
 * loss[i] = (1/n) * sum_b ||x_b - y_mate_b(b)||^2 (float32 of a binary64 sum
 * in a fixed order). Enqueues only. The plan being (1/n) times the
 * permutation, this is its transport cost (the paper motivates using the
 * plan in learning, Section 1). */
int prot_ot_loss_fwd(prot_ctx *ctx, int32_t batch, int64_t n, int32_t d, const float *X,
                     const float *Y, const int32_t *mate_b, float *loss);

/* Its gradient for the fixed matching, for an upstream gradient grad_loss
 * (device float[batch]): dX_b = (2 g / n)(x_b - y_a), dY_a = (2 g / n)(y_a - x_b)
 * for each matched pair mate_b[b] = a, 0 for unmatched points. mate_b must
 * be a matching (no column twice). dX, dY: device, the layout of X, Y.
 * Enqueues only. */
int prot_ot_loss_bwd(prot_ctx *ctx, int32_t batch, int64_t n, int32_t d, const float *X,
                     const float *Y, const int32_t *mate_b, const float *grad_loss, float *dX,
                     float *dY);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): prot_ot_loss_fwd
 * without a context. Same arguments, layout and result (bit for bit); the
 * work is enqueued on hip_stream (a hipStream_t, NULL = the null stream) of
 * the device current on the calling thread. Its partial sums live in a fixed
 * device array of the library, 65,536 doubles (512 KiB) per device, held
 * until the process ends (its address is looked up on the first call on a
 * device); nothing is allocated or freed, and no partial sum needs clearing
 * (every call writes all it reads). Every call on one device shares that
 * array: calls that overlap in time on one GPU (other streams, other
 * threads) race. Errors: PROT_E_ARG (bad pointer or size),
 * PROT_E_UNSUPPORTED when batch x ceil(n d / 8192) (at most 64 per
 * instance) exceeds 65,536 partial sums, PROT_E_HIP; the message is
 * prot_last_error(NULL) on the calling thread. Enqueues only. */
int prot_ot_loss_fwd_static(int32_t batch, int64_t n, int32_t d, const float *X, const float *Y,
                            const int32_t *mate_b, float *loss, void *hip_stream);

const char *prot_status_string(int status);
/* The message of ctx's last failed call; with ctx = NULL, that of the last
 * failed context-free call on this thread ("null context" if none). */
const char *prot_last_error(prot_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
