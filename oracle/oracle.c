/*
 * CPU oracle for the push-relabel additive epsilon-approximation of the
 * assignment problem (arXiv:2203.03732). TEST INFRASTRUCTURE: see oracle.h.
 *
 * Plain single-threaded C, written from the paper's description of the
 * algorithm (Section 2.2) and its sequential realisation (proof of
 * Lemma 3.4). Nothing here is tuned; every step is done in the order the
 * paper states it. Where the paper leaves a choice open, the reading used
 * is stated at the point where the choice is made.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Section 2.1, eq. (1): cbar(a, b) = eps * floor(c(a, b) / eps).       */
/* Costs are assumed scaled so that the largest one is 1 (Section 1), */
/* so a cost outside [0, 1] (or NaN) is rejected.                     */
/* ------------------------------------------------------------------ */

static int eps_ok(double eps)
{
    if (!(eps > 0.0 && eps < 1.0)) return 0;
    /* the largest rounded cost plus the two dual steps must fit int16 */
    if (floor(1.0 / eps) + 2.0 > 32767.0) return 0;
    return 1;
}

int orc_round_cost(const float *C, int64_t n_b, int64_t n_a, int64_t ldc,
                   double eps, int16_t *k, int64_t ldk)
{
    if (!C || !k || n_b < 0 || n_a < 0 || ldc < n_a || ldk < n_a)
        return ORC_E_ARG;
    if (!eps_ok(eps)) return ORC_E_EPS;
    for (int64_t b = 0; b < n_b; ++b) {
        for (int64_t a = 0; a < n_a; ++a) {
            double c = (double)C[b * ldc + a];
            if (!(c >= 0.0 && c <= 1.0)) return ORC_E_RANGE;
            k[b * ldk + a] = (int16_t)floor(c / eps);
        }
    }
    return ORC_OK;
}

int orc_round_points_f32(const float *X, const float *Y, int64_t n_b,
                         int64_t n_a, int32_t d, double eps, int16_t *k,
                         int64_t ldk, float *m_out)
{
    if (!X || !Y || !k || n_b < 0 || n_a < 0 || d <= 0 || ldk < n_a)
        return ORC_E_ARG;
    if (!eps_ok(eps)) return ORC_E_EPS;
    float *d2 = (float *)malloc(sizeof(float) * (size_t)(n_b * n_a + 1));
    if (!d2) return ORC_E_NOMEM;
    float m = 0.0f;
    for (int64_t b = 0; b < n_b; ++b) {
        for (int64_t a = 0; a < n_a; ++a) {
            float s = 0.0f;
            for (int32_t j = 0; j < d; ++j) {
                float t = X[b * d + j] - Y[a * d + j];
                s = fmaf(t, t, s);
            }
            d2[b * n_a + a] = s;
            if (s > m) m = s;
        }
    }
    for (int64_t b = 0; b < n_b; ++b) {
        for (int64_t a = 0; a < n_a; ++a) {
            if (m == 0.0f) {
                k[b * ldk + a] = 0;
            } else {
                double c = (double)d2[b * n_a + a] / (double)m;
                k[b * ldk + a] = (int16_t)floor(c / eps);
            }
        }
    }
    if (m_out) *m_out = m;
    free(d2);
    return ORC_OK;
}

/* Section 5's synthetic cost: the plain Euclidean distance. Same binary32
 * squared distance d2 and maximum m as orc_round_points_f32; the cost scaled
 * to max 1 is sqrt(d2 / m) (division and square root in binary64) and
 * k = floor(c / eps). */
int orc_round_points_euclid_f32(const float *X, const float *Y, int64_t n_b, int64_t n_a,
                                int32_t d, double eps, int16_t *k, int64_t ldk, float *m_out)
{
    if (!X || !Y || !k || n_b < 0 || n_a < 0 || d <= 0 || ldk < n_a)
        return ORC_E_ARG;
    if (!eps_ok(eps)) return ORC_E_EPS;
    float *d2 = (float *)malloc(sizeof(float) * (size_t)(n_b * n_a + 1));
    if (!d2) return ORC_E_NOMEM;
    float m = 0.0f;
    for (int64_t b = 0; b < n_b; ++b)
        for (int64_t a = 0; a < n_a; ++a) {
            float s = 0.0f;
            for (int32_t j = 0; j < d; ++j) {
                float t = X[b * d + j] - Y[a * d + j];
                s = fmaf(t, t, s);
            }
            d2[b * n_a + a] = s;
            if (s > m) m = s;
        }
    for (int64_t b = 0; b < n_b; ++b)
        for (int64_t a = 0; a < n_a; ++a) {
            if (m == 0.0f) {
                k[b * ldk + a] = 0;
            } else {
                double c = sqrt((double)d2[b * n_a + a] / (double)m);
                k[b * ldk + a] = (int16_t)floor(c / eps);
            }
        }
    if (m_out) *m_out = m;
    free(d2);
    return ORC_OK;
}

/* Section 5's image cost: each vector is normalised to sum 1 (its sum taken
 * in binary32 in coordinate order, each coordinate divided by it in
 * binary32), and the cost is the L1 distance of the normalised vectors
 * (binary32, coordinate order), at most 2; it is scaled by 1/2 (clamped to 1
 * against rounding) and rounded by eq. (1) in binary64. Entries must be
 * finite and nonnegative with a positive sum. */
int orc_round_l1_normalized_f32(const float *X, const float *Y, int64_t n_b, int64_t n_a,
                                int32_t d, double eps, int16_t *k, int64_t ldk)
{
    if (!X || !Y || !k || n_b < 0 || n_a < 0 || d <= 0 || ldk < n_a)
        return ORC_E_ARG;
    if (!eps_ok(eps)) return ORC_E_EPS;
    float *xh = (float *)malloc(sizeof(float) * (size_t)(n_b * d + 1));
    float *yh = (float *)malloc(sizeof(float) * (size_t)(n_a * d + 1));
    if (!xh || !yh) {
        free(xh); free(yh);
        return ORC_E_NOMEM;
    }
    const float *src[2] = {X, Y};
    float *dst[2] = {xh, yh};
    const int64_t cnt[2] = {n_b, n_a};
    for (int w = 0; w < 2; ++w)
        for (int64_t i = 0; i < cnt[w]; ++i) {
            float sum = 0.0f;
            for (int32_t j = 0; j < d; ++j) {
                float v = src[w][i * d + j];
                if (!(v >= 0.0f && v <= 3.4028234663852886e38f)) {
                    free(xh); free(yh);
                    return ORC_E_RANGE;
                }
                sum = sum + v;
            }
            if (!(sum > 0.0f && sum <= 3.4028234663852886e38f)) {
                free(xh); free(yh);
                return ORC_E_RANGE;
            }
            for (int32_t j = 0; j < d; ++j) dst[w][i * d + j] = src[w][i * d + j] / sum;
        }
    for (int64_t b = 0; b < n_b; ++b)
        for (int64_t a = 0; a < n_a; ++a) {
            float t = 0.0f;
            for (int32_t j = 0; j < d; ++j) t = t + fabsf(xh[b * d + j] - yh[a * d + j]);
            double c = (double)t * 0.5;
            if (c > 1.0) c = 1.0;
            k[b * ldk + a] = (int16_t)floor(c / eps);
        }
    free(xh);
    free(yh);
    return ORC_OK;
}

/* The same binary32 squared distance as orc_round_points_f32, for large
 * instances whose n^2 matrix is not wanted: the maximum over all pairs, then
 * eq. (1) for chosen pairs (b_i, a_i) only. */
static float sq_f32(const float *x, const float *y, int32_t d)
{
    float s = 0.0f;
    for (int32_t j = 0; j < d; ++j) {
        float t = x[j] - y[j];
        s = fmaf(t, t, s);
    }
    return s;
}

int orc_points_max_f32(const float *X, const float *Y, int64_t n_b, int64_t n_a, int32_t d,
                       float *m_out)
{
    if (!X || !Y || !m_out || n_b < 0 || n_a < 0 || d <= 0) return ORC_E_ARG;
    float m = 0.0f;
    for (int64_t b = 0; b < n_b; ++b)
        for (int64_t a = 0; a < n_a; ++a) {
            float s = sq_f32(X + b * d, Y + a * d, d);
            if (s > m) m = s;
        }
    *m_out = m;
    return ORC_OK;
}

int orc_points_pairs_f32(const float *X, const float *Y, int32_t d, double eps, float m,
                         const int64_t *b_idx, const int64_t *a_idx, int64_t count,
                         int16_t *k_out)
{
    if (!X || !Y || !b_idx || !a_idx || !k_out || count < 0 || d <= 0) return ORC_E_ARG;
    if (!eps_ok(eps)) return ORC_E_EPS;
    for (int64_t i = 0; i < count; ++i) {
        if (m == 0.0f) {
            k_out[i] = 0;
        } else {
            double c = (double)sq_f32(X + b_idx[i] * d, Y + a_idx[i] * d, d) / (double)m;
            k_out[i] = (int16_t)floor(c / eps);
        }
    }
    return ORC_OK;
}

int orc_points_cost_f64(const float *X, const float *Y, int64_t n_b,
                        int64_t n_a, int32_t d, double eps, double *c64,
                        int16_t *k64, double *m_out)
{
    if (!X || !Y || n_b < 0 || n_a < 0 || d <= 0) return ORC_E_ARG;
    if (k64 && !eps_ok(eps)) return ORC_E_EPS;
    double *d2 = (double *)malloc(sizeof(double) * (size_t)(n_b * n_a + 1));
    if (!d2) return ORC_E_NOMEM;
    double m = 0.0;
    for (int64_t b = 0; b < n_b; ++b) {
        for (int64_t a = 0; a < n_a; ++a) {
            double s = 0.0;
            for (int32_t j = 0; j < d; ++j) {
                double t = (double)X[b * d + j] - (double)Y[a * d + j];
                s += t * t;
            }
            d2[b * n_a + a] = s;
            if (s > m) m = s;
        }
    }
    for (int64_t i = 0; i < n_b * n_a; ++i) {
        double c = (m == 0.0) ? 0.0 : d2[i] / m;
        if (c64) c64[i] = c;
        if (k64) k64[i] = (int16_t)floor(c / eps);
    }
    if (m_out) *m_out = m;
    free(d2);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Section 2.2: the phase loop.                                        */
/* ------------------------------------------------------------------ */

/* Column visited at step j of the scan of row b. The paper lets a free b
 * take the first admissible edge it meets (proof of Lemma 3.4) without
 * fixing the order in which it looks. Reading used here: DIAG starts row b at column b and wraps around,
 * ZERO starts every row at column 0. */
static int64_t scan_col(int32_t origin_mode, int64_t b, int64_t j, int64_t n)
{
    if (origin_mode == ORC_ORIGIN_ZERO) return j;
    int64_t a = b + j;
    return a >= n ? a - n : a;
}

/* The rounded cost of edge (a, b). Plain instances read k[b][a]. The copies
 * of the transport reduction (Section 4) read the cost of the points they
 * copy: row_pt[b] and col_pt[a] name those points. Point sets given without
 * a matrix (k NULL) compute eq. (1) of the pair from the points each time:
 * the binary32 squared distance of orc_round_points_f32, divided by the
 * maximum m and then by eps in binary64, floored (0 everywhere if m = 0). */
typedef struct {
    const int16_t *k;
    int64_t ldk;
    const int32_t *row_pt, *col_pt;  /* NULL: the identity */
    const float *X, *Y;              /* used when k is NULL */
    int32_t d;
    float m;
    double eps;
} costs_t;

static int16_t cost_of(const costs_t *c, int64_t b, int64_t a)
{
    int64_t r = c->row_pt ? c->row_pt[b] : b;
    int64_t q = c->col_pt ? c->col_pt[a] : a;
    if (!c->k) {
        if (c->m == 0.0f) return 0;
        double v = (double)sq_f32(c->X + r * c->d, c->Y + q * c->d, c->d) / (double)c->m;
        return (int16_t)floor(v / c->eps);
    }
    return c->k[r * c->ldk + q];
}

/* An edge (a, b) outside M is admissible when its slack is zero. With the
 * duals and costs in units of eps, the reading that makes the proof of (I2)
 * go through (a new M' edge must end with y(a) + y(b) = cbar after y(a)
 * drops by one step) is y(a) + y(b) = cbar(a, b) + eps. */
static int admissible_c(const costs_t *c, const int32_t *y_a, const int32_t *y_b, int64_t a,
                        int64_t b)
{
    return (int64_t)cost_of(c, b, a) + 1 == (int64_t)y_a[a] + (int64_t)y_b[b];
}

/* The phase loop on n_b rows and n_a >= n_b columns. With raise_groups > 0
 * (the copies of Section 4) row b is a copy of supply point cs->row_pt[b]
 * and, after step (III) of every phase, each free copy's dual is raised to
 * the largest dual among the copies of its point. */
static int phase_loop(const costs_t *cs, int64_t n_b, int64_t n_a, int64_t raise_groups,
                      int64_t T, int32_t origin_mode, int64_t max_phases, int32_t warm,
                      int32_t complete, int32_t *mate_a, int32_t *mate_b,
                      int32_t *y_a, int32_t *y_b, orc_stats *st,
                      int64_t *trace, int64_t trace_cap)
{
    if (origin_mode != ORC_ORIGIN_DIAG && origin_mode != ORC_ORIGIN_ZERO)
        return ORC_E_ARG;
    memset(st, 0, sizeof(*st));

    /* Initialisation: y(b) = eps, y(a) = 0, M empty. */
    if (!warm) {
        for (int64_t b = 0; b < n_b; ++b) {
            y_b[b] = 1;
            mate_b[b] = -1;
        }
        for (int64_t a = 0; a < n_a; ++a) {
            y_a[a] = 0;
            mate_a[a] = -1;
        }
    }

    size_t sz = (size_t)(n_a > 0 ? n_a : 1);  /* n_b <= n_a */
    int32_t *group_max = NULL;
    if (raise_groups > 0) {
        group_max = (int32_t *)malloc(sizeof(int32_t) * (size_t)raise_groups);
        if (!group_max) return ORC_E_NOMEM;
    }
    int64_t *B_prime = (int64_t *)malloc(sizeof(int64_t) * sz);
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * sz);
    int64_t *target = (int64_t *)malloc(sizeof(int64_t) * sz);
    char *active = (char *)malloc(sz);
    char *won = (char *)malloc(sz);
    int64_t *taken_by = (int64_t *)malloc(sizeof(int64_t) * sz);
    int64_t *proposer = (int64_t *)malloc(sizeof(int64_t) * sz);
    if (!B_prime || !pos || !target || !active || !won || !taken_by ||
        !proposer) {
        free(B_prime); free(pos); free(target); free(active); free(won);
        free(taken_by); free(proposer); free(group_max);
        return ORC_E_NOMEM;
    }

    int status = ORC_OK;
    for (;;) {
        /* B' = the free vertices of B, in ascending order. */
        int64_t n_i = 0;
        for (int64_t b = 0; b < n_b; ++b)
            if (mate_b[b] < 0) B_prime[n_i++] = b;

        /* Stop once |B'| <= eps |B| (integer threshold T). */
        if (n_i <= T) break;
        if (max_phases > 0 && st->phases == max_phases) {
            status = ORC_PARTIAL;
            break;
        }
        st->phases += 1;
        st->sum_free += n_i;
        int64_t phase_scanned = 0, phase_rounds = 0, phase_matched = 0;

        /* Step (I): a maximal matching M' on the admissible edges incident
         * on B'. The paper allows any maximal matching. Reading used here:
         * synchronous proposal rounds. In each round every b of B' that is
         * still looking proposes to the first column in its scan order that
         * is admissible and was not taken before the round began; every
         * column proposed to goes to its lowest-index proposer; losers go on
         * scanning after the column they lost. A b that finds nothing stays
         * free in M'. */
        for (int64_t a = 0; a < n_a; ++a) taken_by[a] = -1;
        for (int64_t i = 0; i < n_i; ++i) {
            pos[i] = 0;
            active[i] = 1;
            won[i] = 0;
        }
        for (;;) {
            int64_t proposals = 0;
            /* (i) propose, against the taken set of the start of the round */
            for (int64_t i = 0; i < n_i; ++i) {
                if (!active[i]) continue;
                int64_t b = B_prime[i];
                target[i] = -1;
                int64_t j;
                for (j = pos[i]; j < n_a; ++j) {
                    int64_t a = scan_col(origin_mode, b, j, n_a);
                    if (taken_by[a] < 0 && admissible_c(cs, y_a, y_b, a, b)) {
                        target[i] = a;
                        break;
                    }
                }
                if (target[i] < 0) {
                    phase_scanned += n_a - pos[i];
                    active[i] = 0; /* no admissible free column is left */
                } else {
                    phase_scanned += j - pos[i] + 1;
                    pos[i] = j;
                    proposals += 1;
                }
            }
            if (proposals == 0) break;
            /* (ii) each proposed-to column goes to its lowest-index proposer */
            for (int64_t i = 0; i < n_i; ++i)
                if (active[i]) proposer[target[i]] = -1;
            for (int64_t i = 0; i < n_i; ++i) {
                if (!active[i]) continue;
                int64_t a = target[i], b = B_prime[i];
                if (proposer[a] < 0 || b < proposer[a]) proposer[a] = b;
            }
            /* (iii) winners take their column; losers resume one further */
            for (int64_t i = 0; i < n_i; ++i) {
                if (!active[i]) continue;
                int64_t a = target[i];
                if (proposer[a] == B_prime[i]) {
                    taken_by[a] = B_prime[i];
                    won[i] = 1;
                    active[i] = 0;
                    phase_matched += 1;
                } else {
                    pos[i] += 1;
                }
            }
            phase_rounds += 1;
        }

        /* Step (II): add M' to M and delete the M-edges of the columns that
         * M' re-matches (the set A'' and its edges M''). */
        for (int64_t a = 0; a < n_a; ++a) {
            int64_t b = taken_by[a];
            if (b < 0) continue;
            if (mate_a[a] >= 0) mate_b[mate_a[a]] = -1;
            mate_a[a] = (int32_t)b;
            mate_b[b] = (int32_t)a;
        }
        /* Step (III a): y(a) -= eps for every edge (a, b) of M'. */
        for (int64_t a = 0; a < n_a; ++a)
            if (taken_by[a] >= 0) y_a[a] -= 1;
        /* Step (III b): y(b) += eps for every b of B' left free by M'. */
        for (int64_t i = 0; i < n_i; ++i)
            if (!won[i]) y_b[B_prime[i]] += 1;

        /* Section 4: every free copy takes the largest dual among the copies
         * of its point (the duals of the copies only grow, and a free copy
         * raised to a sibling's dual keeps eq. (2): the copies share one
         * row of costs). */
        if (raise_groups > 0) {
            for (int64_t g = 0; g < raise_groups; ++g) group_max[g] = INT32_MIN;
            for (int64_t b = 0; b < n_b; ++b) {
                int32_t g = cs->row_pt[b];
                if (y_b[b] > group_max[g]) group_max[g] = y_b[b];
            }
            for (int64_t b = 0; b < n_b; ++b)
                if (mate_b[b] < 0 && y_b[b] < group_max[cs->row_pt[b]])
                    y_b[b] = group_max[cs->row_pt[b]];
        }

        st->rounds += phase_rounds;
        if (phase_rounds > st->max_rounds) st->max_rounds = phase_rounds;
        st->scanned += phase_scanned;
        if (trace && st->phases <= trace_cap) {
            int64_t *t = trace + 4 * (st->phases - 1);
            t[0] = n_i;
            t[1] = phase_rounds;
            t[2] = phase_scanned;
            t[3] = phase_matched;
        }
    }

    int64_t matched = 0;
    for (int64_t b = 0; b < n_b; ++b)
        if (mate_b[b] >= 0) matched += 1;
    st->matched_in_phases = matched;

    /* Completion (Section 2.1): match the remaining free vertices
     * arbitrarily. Reading used here: the i-th free b (ascending) takes the
     * i-th free a (ascending). */
    if (complete && status == ORC_OK) {
        int64_t ia = 0;
        for (int64_t b = 0; b < n_b; ++b) {
            if (mate_b[b] >= 0) continue;
            while (ia < n_a && mate_a[ia] >= 0) ++ia;
            if (ia >= n_a) break;
            mate_b[b] = (int32_t)ia;
            mate_a[ia] = (int32_t)b;
            st->completed_pairs += 1;
        }
    }

    int64_t sum_k = 0;
    for (int64_t b = 0; b < n_b; ++b)
        if (mate_b[b] >= 0) sum_k += cost_of(cs, b, mate_b[b]);
    st->sum_k = sum_k;

    free(B_prime); free(pos); free(target); free(active); free(won);
    free(taken_by); free(proposer); free(group_max);
    return status;
}

int orc_solve_rounded_rect(const int16_t *k, int64_t n_b, int64_t n_a, int64_t ldk,
                           int64_t T, int32_t origin_mode, int64_t max_phases, int32_t warm,
                           int32_t complete, int32_t *mate_a, int32_t *mate_b,
                           int32_t *y_a, int32_t *y_b, orc_stats *st,
                           int64_t *trace, int64_t trace_cap)
{
    if (n_b < 0 || n_a < n_b || (n_b > 0 && (!k || ldk < n_a)) || !mate_a || !mate_b ||
        !y_a || !y_b || !st)
        return ORC_E_ARG;
    costs_t cs = {k, ldk, NULL, NULL, NULL, NULL, 0, 0.0f, 0.0};
    return phase_loop(&cs, n_b, n_a, 0, T, origin_mode, max_phases, warm, complete, mate_a,
                      mate_b, y_a, y_b, st, trace, trace_cap);
}

int orc_solve_points_f32(const float *X, const float *Y, int64_t n_b, int64_t n_a, int32_t d,
                         double eps, int64_t T, int32_t origin_mode, int64_t max_phases,
                         int32_t complete, int32_t *mate_a, int32_t *mate_b, int32_t *y_a,
                         int32_t *y_b, orc_stats *st, int64_t *trace, int64_t trace_cap,
                         float *m_out)
{
    if (!X || !Y || n_b < 0 || n_a < n_b || d <= 0 || !mate_a || !mate_b || !y_a || !y_b ||
        !st)
        return ORC_E_ARG;
    if (!eps_ok(eps)) return ORC_E_EPS;
    float m = 0.0f;
    int rc = orc_points_max_f32(X, Y, n_b, n_a, d, &m);
    if (rc) return rc;
    if (m_out) *m_out = m;
    costs_t cs = {NULL, 0, NULL, NULL, X, Y, d, m, eps};
    return phase_loop(&cs, n_b, n_a, 0, T, origin_mode, max_phases, 0, complete, mate_a,
                      mate_b, y_a, y_b, st, trace, trace_cap);
}

int orc_solve_rounded(const int16_t *k, int64_t n, int64_t ldk, int64_t T,
                      int32_t origin_mode, int64_t max_phases, int32_t warm,
                      int32_t complete, int32_t *mate_a, int32_t *mate_b,
                      int32_t *y_a, int32_t *y_b, orc_stats *st,
                      int64_t *trace, int64_t trace_cap)
{
    return orc_solve_rounded_rect(k, n, n, ldk, T, origin_mode, max_phases, warm, complete,
                                  mate_a, mate_b, y_a, y_b, st, trace, trace_cap);
}

/* ------------------------------------------------------------------ */
/* Section 4: optimal transport through copies.                        */
/* ------------------------------------------------------------------ */

int orc_ot_scale(const double *nu, int64_t n_b, const double *mu, int64_t n_a, double eps,
                 int64_t *s, int64_t *d, double *theta, int64_t *copies_b, int64_t *copies_a)
{
    if (!nu || !mu || n_b < 1 || n_a < 1 || !theta || !copies_b || !copies_a)
        return ORC_E_ARG;
    if (!eps_ok(eps)) return ORC_E_EPS;
    /* the masses are probability vectors */
    double sb = 0.0, sa = 0.0;
    for (int64_t b = 0; b < n_b; ++b) {
        if (!(nu[b] >= 0.0 && nu[b] <= 1.0)) return ORC_E_RANGE;
        sb += nu[b];
    }
    for (int64_t a = 0; a < n_a; ++a) {
        if (!(mu[a] >= 0.0 && mu[a] <= 1.0)) return ORC_E_RANGE;
        sa += mu[a];
    }
    if (fabs(sb - 1.0) > 1e-9 || fabs(sa - 1.0) > 1e-9) return ORC_E_RANGE;
    /* theta = 4n / eps; supplies rounded down, demands rounded up */
    const int64_t n = n_b > n_a ? n_b : n_a;
    const double th = 4.0 * (double)n / eps;
    int64_t cb = 0, ca = 0;
    for (int64_t b = 0; b < n_b; ++b) {
        int64_t v = (int64_t)floor(th * nu[b]);
        if (s) s[b] = v;
        cb += v;
    }
    for (int64_t a = 0; a < n_a; ++a) {
        int64_t v = (int64_t)ceil(th * mu[a]);
        if (d) d[a] = v;
        ca += v;
    }
    if (cb > ca || ca > INT32_MAX) return ORC_E_ARG;
    *theta = th;
    *copies_b = cb;
    *copies_a = ca;
    return ORC_OK;
}

/* The plan of Section 4 from the number of matched pairs of copies between
 * each supply point b and demand point a (cnt, n_b x n_a): every pair carries
 * 1/theta. Then the feasibility repair (the paper leaves it implicit): a
 * demand point that received more than mu_a (its copies were rounded up)
 * gives the excess back, taken from its edges in ascending b, and the mass
 * still to be sent (what the rounding down of the supplies kept back, plus
 * the excess) is paired with the room left at the demand points in order of
 * index (north-west corner rule on the running totals). r and q are scratch
 * of n_b + 1 and n_a + 1 entries. Writes info[1] (cost) and info[2] (mass
 * moved by the repair). */
static void plan_from_counts(const int64_t *cnt, const float *C, int64_t ldc, int64_t n_b,
                             int64_t n_a, const double *nu, const double *mu, double theta,
                             double *plan, double *r, double *q, double *info)
{
    for (int64_t i = 0; i < n_b * n_a; ++i) plan[i] = (double)cnt[i] / theta;
    for (int64_t a = 0; a < n_a; ++a) {
        int64_t c_a = 0;
        for (int64_t b = 0; b < n_b; ++b) c_a += cnt[b * n_a + a];
        double ex = (double)c_a / theta - mu[a];
        for (int64_t b = 0; b < n_b && ex > 0.0; ++b) {
            double v = plan[b * n_a + a];
            if (v <= 0.0) continue;
            double take = v < ex ? v : ex;
            plan[b * n_a + a] = v - take;
            ex = ex - take;
        }
    }
    /* what each supply point still has to send, and the room each demand
     * point has left ... */
    r[0] = 0.0;
    for (int64_t b = 0; b < n_b; ++b) {
        double sent = 0.0;
        for (int64_t a = 0; a < n_a; ++a) sent += plan[b * n_a + a];
        double left = nu[b] - sent;
        r[b + 1] = r[b] + (left > 0.0 ? left : 0.0);
    }
    q[0] = 0.0;
    for (int64_t a = 0; a < n_a; ++a) {
        double got = 0.0;
        for (int64_t b = 0; b < n_b; ++b) got += plan[b * n_a + a];
        double room = mu[a] - got;
        q[a + 1] = q[a] + (room > 0.0 ? room : 0.0);
    }
    /* ... are paired in order: supply b's share [r_b, r_{b+1}) of the
     * running total meets demand a's [q_a, q_{a+1}). */
    for (int64_t b = 0; b < n_b; ++b)
        for (int64_t a = 0; a < n_a; ++a) {
            double lo = r[b] > q[a] ? r[b] : q[a];
            double hi = r[b + 1] < q[a + 1] ? r[b + 1] : q[a + 1];
            if (hi > lo) plan[b * n_a + a] += hi - lo;
        }
    double cost = 0.0;
    for (int64_t b = 0; b < n_b; ++b)
        for (int64_t a = 0; a < n_a; ++a) cost += plan[b * n_a + a] * (double)C[b * ldc + a];
    info[1] = cost;
    info[2] = r[n_b];
}

int orc_ot_solve(const float *C, int64_t n_b, int64_t n_a, int64_t ldc, const double *nu,
                 const double *mu, double eps, int32_t origin_mode, int64_t max_phases,
                 int32_t warm, int32_t *mate_a, int32_t *mate_b, int32_t *y_a, int32_t *y_b,
                 double *plan, orc_stats *st, double *info, int64_t *trace, int64_t trace_cap)
{
    if (!C || ldc < n_a || !mate_a || !mate_b || !y_a || !y_b || !plan || !st || !info)
        return ORC_E_ARG;
    double theta = 0.0;
    int64_t NB = 0, NA = 0;
    int64_t *s = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_b > 0 ? n_b : 1));
    int64_t *d = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_a > 0 ? n_a : 1));
    if (!s || !d) {
        free(s); free(d);
        return ORC_E_NOMEM;
    }
    int rc = orc_ot_scale(nu, n_b, mu, n_a, eps, s, d, &theta, &NB, &NA);
    if (rc) {
        free(s); free(d);
        return rc;
    }
    /* the copies: supply point b owns rows [sum_{b'<b} s_b', ...), demand
     * point a owns columns [sum_{a'<a} d_a', ...) */
    int32_t *row_pt = (int32_t *)malloc(sizeof(int32_t) * (size_t)(NB > 0 ? NB : 1));
    int32_t *col_pt = (int32_t *)malloc(sizeof(int32_t) * (size_t)(NA > 0 ? NA : 1));
    int16_t *k = (int16_t *)malloc(sizeof(int16_t) * (size_t)(n_b * n_a));
    int64_t *cnt = (int64_t *)calloc((size_t)(n_b * n_a), sizeof(int64_t));
    double *r = (double *)malloc(sizeof(double) * (size_t)(n_b + 1));
    double *q = (double *)malloc(sizeof(double) * (size_t)(n_a + 1));
    if (!row_pt || !col_pt || !k || !cnt || !r || !q) {
        rc = ORC_E_NOMEM;
        goto out;
    }
    for (int64_t b = 0, i = 0; b < n_b; ++b)
        for (int64_t c = 0; c < s[b]; ++c) row_pt[i++] = (int32_t)b;
    for (int64_t a = 0, i = 0; a < n_a; ++a)
        for (int64_t c = 0; c < d[a]; ++c) col_pt[i++] = (int32_t)a;

    /* eq. (1) on the points' costs; every copy inherits its point's row */
    rc = orc_round_cost(C, n_b, n_a, ldc, eps, k, n_a);
    if (rc) goto out;

    /* the unbalanced matching of the copies (Section 3.3) with the free-copy
     * raise of Section 4; stop at |B'| <= eps |B copies| */
    const int64_t T = (int64_t)floor(eps * (double)NB + 1e-9);
    costs_t cs = {k, n_a, row_pt, col_pt};
    rc = phase_loop(&cs, NB, NA, n_b, T, origin_mode, max_phases, warm, 1, mate_a, mate_b,
                    y_a, y_b, st, trace, trace_cap);
    info[0] = theta;
    info[1] = 0.0;
    info[2] = 0.0;
    info[3] = (double)T;
    if (rc != ORC_OK) goto out;

    /* The plan: every matched pair of copies carries 1/theta. */
    for (int64_t b = 0; b < NB; ++b)
        if (mate_b[b] >= 0) cnt[row_pt[b] * n_a + col_pt[mate_b[b]]] += 1;
    plan_from_counts(cnt, C, ldc, n_b, n_a, nu, mu, theta, plan, r, q, info);

out:
    free(s); free(d); free(row_pt); free(col_pt); free(k); free(cnt); free(r); free(q);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Section 4 with Lemma 4.1: the copies kept as two clusters per point. */
/* ------------------------------------------------------------------ */

/* The level (dual in eps steps) of the demand copies of point a stored in
 * parity slot p: its two levels Z_a and Z_a - 1 differ in parity. */
static int32_t a_level(int32_t Z, int32_t p)
{
    return ((Z & 1) == p) ? Z : Z - 1;
}

/* Lemma 4.1 and eqs. (1)-(2) on the clusters: every matched pair is tight
 * (its supply copy sits at k - its demand copy's level), and that level is
 * Y_b or Y_b - 1; a point with free demand copies has its top at 0. */
static int clusters_ok(const int16_t *k, int64_t ldk, int64_t n_b, int64_t n_a,
                       const int32_t *Y, const int32_t *Z, const int64_t *G, const int64_t *w)
{
    for (int64_t a = 0; a < n_a; ++a)
        if (G[a] > 0 && Z[a] != 0) return 0;
    for (int64_t b = 0; b < n_b; ++b)
        for (int64_t a = 0; a < n_a; ++a)
            for (int32_t p = 0; p < 2; ++p) {
                if (w[(b * n_a + a) * 2 + p] == 0) continue;
                int64_t yb = (int64_t)k[b * ldk + a] - a_level(Z[a], p);
                if (yb != Y[b] && yb != (int64_t)Y[b] - 1) return 0;
            }
    return 1;
}

int orc_ot_clustered_rounded(const int16_t *k, int64_t n_b, int64_t n_a, int64_t ldk,
                             const int64_t *s, const int64_t *d, int64_t T,
                             int32_t origin_mode, int64_t max_phases, int32_t warm,
                             int32_t complete, int32_t *Y, int64_t *F, int32_t *Z, int64_t *G,
                             int64_t *w, int64_t *flow, int64_t *m_last, orc_stats *st,
                             int64_t *trace, int64_t trace_cap)
{
    if (!k || n_b < 1 || n_a < 1 || ldk < n_a || !s || !d || T < 0 || !Y || !F || !Z ||
        !G || !w || !st)
        return ORC_E_ARG;
    if (origin_mode != ORC_ORIGIN_DIAG && origin_mode != ORC_ORIGIN_ZERO) return ORC_E_ARG;
    int64_t NB = 0, NA = 0;
    for (int64_t b = 0; b < n_b; ++b) {
        if (s[b] < 0) return ORC_E_ARG;
        NB += s[b];
    }
    for (int64_t a = 0; a < n_a; ++a) {
        if (d[a] < 0) return ORC_E_ARG;
        NA += d[a];
    }
    if (NB > NA) return ORC_E_ARG;
    memset(st, 0, sizeof(*st));

    /* Initialisation: every supply copy free at y = eps, every demand copy
     * free at 0, no pairs. */
    if (!warm) {
        for (int64_t b = 0; b < n_b; ++b) {
            Y[b] = 1;
            F[b] = s[b];
        }
        for (int64_t a = 0; a < n_a; ++a) {
            Z[a] = 0;
            G[a] = d[a];
        }
        memset(w, 0, sizeof(int64_t) * (size_t)(n_b * n_a * 2));
    }

    int64_t *top = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_a);
    int64_t *cap = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_a);
    int64_t *want = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_b);
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_b);
    int64_t *target = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_b);
    int64_t *evicted = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_b);
    char *active = (char *)malloc((size_t)n_b);
    int64_t *m = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_b * n_a));
    if (!top || !cap || !want || !pos || !target || !evicted || !active || !m) {
        free(top); free(cap); free(want); free(pos); free(target); free(evicted);
        free(active); free(m);
        return ORC_E_NOMEM;
    }

    int status = ORC_OK;
    if (m_last) memset(m_last, 0, sizeof(int64_t) * (size_t)(n_b * n_a));
    for (;;) {
        /* |B'|: the free supply copies */
        int64_t n_free = 0;
        for (int64_t b = 0; b < n_b; ++b) n_free += F[b];
        if (n_free <= T) break;
        if (max_phases > 0 && st->phases == max_phases) {
            status = ORC_PARTIAL;
            break;
        }
        st->phases += 1;
        st->sum_free += n_free;
        int64_t phase_scanned = 0, phase_rounds = 0, phase_matched = 0;

        /* Step (I) on the clusters. The free copies of b all sit at Y_b (the
         * raise), the copies of a at Z_a or Z_a - 1. Edge (a, b) is
         * admissible when k + 1 = Z_a + Y_b; the lower level of a never is,
         * as (I1) on the upper level's copies gives Z_a + Y_b <= k + 1. So a
         * offers its top-level copies: the free ones (top = 0) and those
         * matched at Z_a. Reading used here: point-level synchronous rounds.
         * Every b with copies still looking proposes to the first point in
         * its scan order (DIAG: from column b mod n_a, as supply points may
         * outnumber demand points) that is admissible and had top copies left when the
         * round began, asking for all its looking copies; each point serves
         * its proposers in ascending b, each as far as its copies go; a b
         * served in part, or not at all, goes on scanning after that point.
         * A b that finds nothing keeps its remaining copies free in M'. */
        for (int64_t a = 0; a < n_a; ++a) {
            int64_t t = (Z[a] == 0) ? G[a] : 0;
            for (int64_t b = 0; b < n_b; ++b) t += w[(b * n_a + a) * 2 + (Z[a] & 1)];
            top[a] = t;
            cap[a] = t;
        }
        for (int64_t b = 0; b < n_b; ++b) {
            want[b] = F[b];
            pos[b] = 0;
            active[b] = F[b] > 0;
            evicted[b] = 0;
        }
        memset(m, 0, sizeof(int64_t) * (size_t)(n_b * n_a));
        for (;;) {
            int64_t proposals = 0;
            /* (i) propose, against the top copies left at the round's start */
            for (int64_t b = 0; b < n_b; ++b) {
                if (!active[b]) continue;
                target[b] = -1;
                int64_t j;
                for (j = pos[b]; j < n_a; ++j) {
                    int64_t a = scan_col(origin_mode, b % n_a, j, n_a);
                    if (cap[a] > 0 && (int64_t)k[b * ldk + a] + 1 == (int64_t)Z[a] + Y[b]) {
                        target[b] = a;
                        break;
                    }
                }
                if (target[b] < 0) {
                    phase_scanned += n_a - pos[b];
                    active[b] = 0;
                } else {
                    phase_scanned += j - pos[b] + 1;
                    pos[b] = j;
                    proposals += 1;
                }
            }
            if (proposals == 0) break;
            /* (ii) each point serves its proposers in ascending b */
            for (int64_t b = 0; b < n_b; ++b) {
                if (!active[b]) continue;
                int64_t a = target[b];
                int64_t g = want[b] < cap[a] ? want[b] : cap[a];
                want[b] -= g;
                cap[a] -= g;
                m[b * n_a + a] += g;
                phase_matched += g;
                if (want[b] == 0)
                    active[b] = 0;
                else
                    pos[b] += 1;  /* the point has no top copies left */
            }
            phase_rounds += 1;
        }

        /* Step (II): each point a hands out the top copies M' took: the free
         * ones first, then those matched at Z_a in ascending order of their
         * partner's point, whose partner copies become free (A'' and M''). The
         * taken copies form the new pairs; after (III a) they sit at Z_a - 1,
         * and a point whose top copies are all taken has Z_a - 1 as its top. */
        for (int64_t a = 0; a < n_a; ++a) {
            int64_t taken = top[a] - cap[a];
            if (taken == 0) continue;
            int32_t p = Z[a] & 1;
            if (Z[a] == 0) {
                int64_t u = taken < G[a] ? taken : G[a];
                G[a] -= u;
                taken -= u;
            }
            for (int64_t b = 0; b < n_b && taken > 0; ++b) {
                int64_t *x = &w[(b * n_a + a) * 2 + p];
                int64_t v = taken < *x ? taken : *x;
                *x -= v;
                evicted[b] += v;
                taken -= v;
            }
            int32_t q = (Z[a] - 1) & 1;
            for (int64_t b = 0; b < n_b; ++b) w[(b * n_a + a) * 2 + q] += m[b * n_a + a];
            if (cap[a] == 0) Z[a] -= 1;  /* step (III a) for the whole top */
        }
        /* Step (III b) and the raise: copies of b left free by M' go up one
         * step, so Y_b grows by one when there are any; the evicted copies
         * are free again and take the largest dual of their point, Y_b. */
        for (int64_t b = 0; b < n_b; ++b) {
            if (want[b] > 0) Y[b] += 1;
            F[b] = want[b] + evicted[b];
        }
        if (!clusters_ok(k, ldk, n_b, n_a, Y, Z, G, w)) {
            status = ORC_E_STATE;
            break;
        }
        if (m_last) memcpy(m_last, m, sizeof(int64_t) * (size_t)(n_b * n_a));

        st->rounds += phase_rounds;
        if (phase_rounds > st->max_rounds) st->max_rounds = phase_rounds;
        st->scanned += phase_scanned;
        if (trace && st->phases <= trace_cap) {
            int64_t *t = trace + 4 * (st->phases - 1);
            t[0] = n_free;
            t[1] = phase_rounds;
            t[2] = phase_scanned;
            t[3] = phase_matched;
        }
    }

    int64_t matched = 0, sum_k = 0;
    for (int64_t b = 0; b < n_b; ++b)
        for (int64_t a = 0; a < n_a; ++a) {
            int64_t c = w[(b * n_a + a) * 2] + w[(b * n_a + a) * 2 + 1];
            matched += c;
            sum_k += c * (int64_t)k[b * ldk + a];
            if (flow) flow[b * n_a + a] = c;
        }
    st->matched_in_phases = matched;

    /* Completion: the free supply copies, in order of their point, take the
     * free demand copies in order of theirs (north-west corner rule on the
     * counts F and G; with one copy per point this is the i-th free b taking
     * the i-th free a). The clusters are left as the phase loop ended. */
    if (complete && status == ORC_OK) {
        int64_t a = 0, g = n_a > 0 ? G[0] : 0;
        for (int64_t b = 0; b < n_b; ++b) {
            int64_t f = F[b];
            while (f > 0) {
                while (g == 0 && a + 1 < n_a) g = G[++a];
                if (g == 0) break;
                int64_t v = f < g ? f : g;
                if (flow) flow[b * n_a + a] += v;
                sum_k += v * (int64_t)k[b * ldk + a];
                st->completed_pairs += v;
                f -= v;
                g -= v;
            }
        }
    }
    st->sum_k = sum_k;

    free(top); free(cap); free(want); free(pos); free(target); free(evicted);
    free(active); free(m);
    return status;
}

int orc_ot_solve_clustered(const float *C, int64_t n_b, int64_t n_a, int64_t ldc,
                           const double *nu, const double *mu, double eps, int32_t origin_mode,
                           int64_t max_phases, int32_t warm, int32_t *Y, int64_t *F, int32_t *Z,
                           int64_t *G, int64_t *w, double *plan, orc_stats *st, double *info,
                           int64_t *trace, int64_t trace_cap)
{
    if (!C || ldc < n_a || !Y || !F || !Z || !G || !w || !plan || !st || !info)
        return ORC_E_ARG;
    double theta = 0.0;
    int64_t NB = 0, NA = 0;
    int64_t *s = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_b > 0 ? n_b : 1));
    int64_t *d = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_a > 0 ? n_a : 1));
    if (!s || !d) {
        free(s); free(d);
        return ORC_E_NOMEM;
    }
    int rc = orc_ot_scale(nu, n_b, mu, n_a, eps, s, d, &theta, &NB, &NA);
    if (rc) {
        free(s); free(d);
        return rc;
    }
    int16_t *k = (int16_t *)malloc(sizeof(int16_t) * (size_t)(n_b * n_a));
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_b * n_a));
    double *r = (double *)malloc(sizeof(double) * (size_t)(n_b + 1));
    double *q = (double *)malloc(sizeof(double) * (size_t)(n_a + 1));
    if (!k || !cnt || !r || !q) {
        rc = ORC_E_NOMEM;
        goto out;
    }
    rc = orc_round_cost(C, n_b, n_a, ldc, eps, k, n_a);
    if (rc) goto out;
    /* the same stop as the explicit copies: |B'| <= eps |B copies| */
    const int64_t T = (int64_t)floor(eps * (double)NB + 1e-9);
    rc = orc_ot_clustered_rounded(k, n_b, n_a, n_a, s, d, T, origin_mode, max_phases, warm, 1,
                                  Y, F, Z, G, w, cnt, NULL, st, trace, trace_cap);
    info[0] = theta;
    info[1] = 0.0;
    info[2] = 0.0;
    info[3] = (double)T;
    if (rc != ORC_OK) goto out;
    plan_from_counts(cnt, C, ldc, n_b, n_a, nu, mu, theta, plan, r, q, info);

out:
    free(s); free(d); free(k); free(cnt); free(r); free(q);
    return rc;
}
