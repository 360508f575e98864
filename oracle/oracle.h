/*
 * CPU oracle for the push-relabel additive epsilon-approximation of the
 * assignment problem (Lahn, Raghvendra and Zhang, "A Push-Relabel Based
 * Additive Approximation for Optimal Transport", arXiv:2203.03732).
 *
 * TEST INFRASTRUCTURE. This library exists only to check the GPU library
 * against a plain, slow, single-threaded reading of the paper. Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark load
 * it. It shares no code, header, table or helper with the GPU library.
 *
 * Units: every dual weight is an integer number of epsilon steps, and every
 * rounded cost k is the integer with cbar = eps * k (Section 2.1, eq. (1)).
 * Matrices are row-major with rows = supply vertices B and columns = demand
 * vertices A; k[b*ldk + a] is the rounded cost of edge (a, b).
 */
#ifndef PROT_ORACLE_H
#define PROT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ORC_OK = 0,
    ORC_PARTIAL = 1,      /* stopped after max_phases phases; state is valid */
    ORC_E_ARG = -1,
    ORC_E_RANGE = -2,     /* a cost is NaN or outside [0, 1] */
    ORC_E_EPS = -3,       /* eps outside (0, 1) or 1/eps too large for int16 */
    ORC_E_NOMEM = -7,
    ORC_E_STATE = -8      /* the clusters broke Lemma 4.1 or eq. (2) (a defect) */
};

enum { ORC_ORIGIN_DIAG = 0, ORC_ORIGIN_ZERO = 1 };

typedef struct {
    int64_t phases;           /* phases executed by this call */
    int64_t sum_free;         /* sum over those phases of |B'| */
    int64_t rounds;           /* proposal rounds that made at least one proposal */
    int64_t max_rounds;       /* most such rounds in one phase */
    int64_t scanned;          /* matrix entries examined by the greedy step */
    int64_t matched_in_phases;/* |M| when the phase loop stopped */
    int64_t completed_pairs;  /* pairs added by the arbitrary completion */
    int64_t sum_k;            /* sum of k over the returned matching */
} orc_stats;

/* eq. (1): k = floor(c / eps), one binary64 division then floor. */
int orc_round_cost(const float *C, int64_t n_b, int64_t n_a, int64_t ldc,
                   double eps, int16_t *k, int64_t ldk);

/* Squared Euclidean cost in binary32, accumulated coordinate by coordinate
 * with a fused multiply-add: s = fma(x_j - y_j, x_j - y_j, s). The maximum
 * over all pairs is m; k = floor((d2 / m) / eps) with both divisions in
 * binary64. If m == 0 every k is 0. Writes m to *m_out. */
int orc_round_points_f32(const float *X, const float *Y, int64_t n_b,
                         int64_t n_a, int32_t d, double eps, int16_t *k,
                         int64_t ldk, float *m_out);

/* Cost variants of Section 5. Euclidean: the same d2 and m as above, cost
 * sqrt(d2 / m) (binary64), k = floor(cost / eps). L1 on normalised vectors:
 * every vector divided by its binary32 sum (coordinate order), cost = half
 * the binary32 L1 distance (coordinate order) clamped to 1, k = floor(cost /
 * eps); entries must be finite, nonnegative, with a positive sum
 * (ORC_E_RANGE otherwise). */
int orc_round_points_euclid_f32(const float *X, const float *Y, int64_t n_b, int64_t n_a,
                                int32_t d, double eps, int16_t *k, int64_t ldk, float *m_out);
int orc_round_l1_normalized_f32(const float *X, const float *Y, int64_t n_b, int64_t n_a,
                                int32_t d, double eps, int16_t *k, int64_t ldk);

/* Large instances: the binary32 maximum squared distance over all pairs, and
 * eq. (1) for the chosen pairs (b_idx[i], a_idx[i]) given that maximum. Same
 * arithmetic as orc_round_points_f32. */
int orc_points_max_f32(const float *X, const float *Y, int64_t n_b, int64_t n_a, int32_t d,
                       float *m_out);
int orc_points_pairs_f32(const float *X, const float *Y, int32_t d, double eps, float m,
                         const int64_t *b_idx, const int64_t *a_idx, int64_t count,
                         int16_t *k_out);

/* Reference squared Euclidean cost in binary64 from the same binary32
 * points: c64 = d2_64 / max d2_64 (optional output, n_b x n_a), and
 * k64 = floor(c64 / eps) (optional). Writes the maximum to *m_out. */
int orc_points_cost_f64(const float *X, const float *Y, int64_t n_b,
                        int64_t n_a, int32_t d, double eps, double *c64,
                        int16_t *k64, double *m_out);

/* The integer phase loop of Section 2.2 followed by the arbitrary completion.
 *   k, ldk      : n x n rounded costs (rows B, columns A)
 *   T           : stop when |B'| <= T (T = floor(eps * n))
 *   origin_mode : where the scan of row b starts (ORC_ORIGIN_*)
 *   max_phases  : stop after this many phases (<= 0: no limit)
 *   warm        : 0 = start from y(b) = 1, y(a) = 0, M empty; 1 = resume
 *                 from the given mate/dual arrays
 *   complete    : 1 = match the last free vertices arbitrarily
 *   mate_a[a]   : b matched to a, or -1; mate_b[b]: a matched to b, or -1
 *   y_a, y_b    : dual weights in units of eps
 *   trace       : optional, 4 int64 per phase (|B'|, rounds, scanned, |M'|)
 * Returns ORC_OK, ORC_PARTIAL (max_phases reached) or an error. */
/* The unbalanced case (Section 3.3): |B| = n_b rows <= |A| = n_a columns,
 * k is n_b x ldk (ldk >= n_a), y_b/mate_b have n_b entries, y_a/mate_a n_a.
 * The loop is unchanged; it stops at |B'| <= T with T = floor(eps n_b), and
 * the completion pairs the i-th free b with the i-th free a. DIAG starts row
 * b at column b (b < n_b <= n_a). */
int orc_solve_rounded_rect(const int16_t *k, int64_t n_b, int64_t n_a, int64_t ldk,
                           int64_t T, int32_t origin_mode, int64_t max_phases, int32_t warm,
                           int32_t complete, int32_t *mate_a, int32_t *mate_b,
                           int32_t *y_a, int32_t *y_b, orc_stats *st,
                           int64_t *trace, int64_t trace_cap);

int orc_solve_rounded(const int16_t *k, int64_t n, int64_t ldk, int64_t T,
                      int32_t origin_mode, int64_t max_phases, int32_t warm,
                      int32_t complete, int32_t *mate_a, int32_t *mate_b,
                      int32_t *y_a, int32_t *y_b, orc_stats *st,
                      int64_t *trace, int64_t trace_cap);

/* The phase loop (as orc_solve_rounded_rect, cold start) on point sets
 * without the n_b x n_a matrix: m = orc_points_max_f32 first, then every
 * rounded cost the loop examines is eq. (1) of that pair with the arithmetic
 * of orc_round_points_f32. Writes m to *m_out (optional). */
int orc_solve_points_f32(const float *X, const float *Y, int64_t n_b, int64_t n_a, int32_t d,
                         double eps, int64_t T, int32_t origin_mode, int64_t max_phases,
                         int32_t complete, int32_t *mate_a, int32_t *mate_b, int32_t *y_a,
                         int32_t *y_b, orc_stats *st, int64_t *trace, int64_t trace_cap,
                         float *m_out);

/* Section 4, scaling: theta = 4 max(n_b, n_a) / eps; supply point b becomes
 * s_b = floor(theta nu_b) unit copies, demand point a d_a = ceil(theta mu_a)
 * (binary64 products). nu and mu are probability vectors (entries in [0, 1],
 * sums within 1e-9 of 1). s and d are optional outputs. */
int orc_ot_scale(const double *nu, int64_t n_b, const double *mu, int64_t n_a, double eps,
                 int64_t *s, int64_t *d, double *theta, int64_t *copies_b, int64_t *copies_a);

/* Section 4: an approximate transport plan from supplies nu (rows of C,
 * n_b points) to demands mu (columns, n_a points), costs C in [0, 1].
 * The copies (rows: supply copies, point b's copies contiguous and in order
 * of b; columns likewise) form an unbalanced matching instance whose
 * rounded cost is eq. (1) of the points' cost. The phase loop runs on it
 * with T = floor(eps |B copies|) and, after step (III) of every phase, each
 * free supply copy's dual is raised to the largest dual among the copies of
 * its point. After the completion every matched pair of copies carries
 * 1/theta from its supply point to its demand point; then (feasibility
 * repair) a demand point holding more than mu_a gives the excess back, taken
 * from its edges in ascending b, and the mass still to be sent (what the
 * rounding down of the supplies kept back, plus the excess) is paired with
 * the room left at the demand points in order of index (north-west corner
 * rule on the running totals).
 *   mate_a, y_a : copies_a entries; mate_b, y_b: copies_b entries (copy level)
 *   plan        : n_b x n_a, row-major (written when the loop finished)
 *   info        : theta, plan cost sum plan * C, mass moved by the repair, T
 * max_phases and warm as for the phase loop (warm resumes from the copy-level
 * arrays); the plan is written only when the loop finished (ORC_OK). */
int orc_ot_solve(const float *C, int64_t n_b, int64_t n_a, int64_t ldc, const double *nu,
                 const double *mu, double eps, int32_t origin_mode, int64_t max_phases,
                 int32_t warm, int32_t *mate_a, int32_t *mate_b, int32_t *y_a, int32_t *y_b,
                 double *plan, orc_stats *st, double *info, int64_t *trace, int64_t trace_cap);

/* Section 4 with Lemma 4.1: the transport copies kept as clusters. Supply
 * point b has s[b] copies, demand point a d[a] (sum s <= sum d); a copy's
 * rounded cost is its points' k. State, all in eps steps:
 *   Y[b] : the largest dual among b's copies; its free copies sit there and
 *          its matched ones at Y[b] or Y[b] - 1
 *   F[b] : b's free copies
 *   Z[a] : the largest dual among a's copies; they sit at Z[a] or Z[a] - 1
 *   G[a] : a's free copies (dual 0; G[a] > 0 only when Z[a] = 0)
 *   w    : n_b x n_a x 2, w[(b*n_a + a)*2 + p] = pairs between copies of b
 *          and copies of a whose demand copy's level has parity p; the
 *          supply copy of such a pair sits at k[b][a] minus that level
 * A phase is steps (I)-(III) of Section 2.2 on the copies with the free-copy
 * raise of Section 4, taken point by point (the reading is stated in the
 * code); phases run while sum F > T. flow (optional, n_b x n_a) receives the
 * pairs per point pair, plus the completion's when complete is set; m_last
 * (optional, n_b x n_a) the pairs M' formed in the last phase. warm resumes
 * from Y, F, Z, G, w. ORC_E_STATE when a check of Lemma 4.1 fails. */
int orc_ot_clustered_rounded(const int16_t *k, int64_t n_b, int64_t n_a, int64_t ldk,
                             const int64_t *s, const int64_t *d, int64_t T,
                             int32_t origin_mode, int64_t max_phases, int32_t warm,
                             int32_t complete, int32_t *Y, int64_t *F, int32_t *Z, int64_t *G,
                             int64_t *w, int64_t *flow, int64_t *m_last, orc_stats *st,
                             int64_t *trace, int64_t trace_cap);

/* orc_ot_solve with the copies kept as clusters (orc_ot_clustered_rounded):
 * same scaling, rounding, stop threshold, completion reading, plan and
 * repair, and the same info. */
int orc_ot_solve_clustered(const float *C, int64_t n_b, int64_t n_a, int64_t ldc,
                           const double *nu, const double *mu, double eps, int32_t origin_mode,
                           int64_t max_phases, int32_t warm, int32_t *Y, int64_t *F, int32_t *Z,
                           int64_t *G, int64_t *w, double *plan, orc_stats *st, double *info,
                           int64_t *trace, int64_t trace_cap);

#ifdef __cplusplus
}
#endif
#endif
