// Host runtime and C ABI of libprot (declarations and contracts: include/prot.h).
//
// A context owns a stream handle, the device workspace of the phase loop
// (per-column keys and duals, the free and taken lists, the control block and
// the phase trace), an optional rounded-cost matrix for the cost and point
// entry points, and a pinned host staging buffer for the statistics. Each
// call validates its arguments, enqueues its kernels on the stream and, if
// it returns statistics, synchronises once at the end.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <string>
#include <vector>

#include "../../include/prot.h"
#include "internal.h"

using prot::Ctl;

// Device block read back in one transfer after a solve: the control block
// and the finalize pass's partial sums.
struct Report {
    Ctl ctl;
    long long part_k[prot::kFinalizeBlocks];
    double part_c[prot::kFinalizeBlocks];
};

struct prot_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;

    int64_t cap_n = 0;               // loop workspace capacity (vertices)
    unsigned long long *key = nullptr;
    uint16_t *t = nullptr;
    int32_t *lists = nullptr;        // completion scratch (2n)
    unsigned long long *tlists = nullptr;  // tagged F0, F1, L0, L1 of the phase loop
    unsigned long long *words = nullptr;   // round words of the phase loop barrier
    Report *rep = nullptr;
    Ctl *ctl = nullptr;              // &rep->ctl
    int64_t *trace = nullptr;
    long long *part_k = nullptr;     // rep->part_k
    double *part_c = nullptr;        // rep->part_c

    int64_t cap_mat = 0;             // elements of the rounded-cost matrix
    int16_t *kmat = nullptr;
    int32_t cap_th = 0;
    float *th = nullptr;
    char *prune_buf = nullptr;       // pruned-maximum workspace (d = 2, 3)
    int64_t prune_cap = 0;
    int64_t prune_min_n = 16384;     // PROT_PRUNE_MIN_N
    float *mpart = nullptr;          // per-block maxima of the maximum pass (d = 2, 3)
    int64_t mpart_cap = 0;

    struct Stage {                   // begins with the layout of Report
        Ctl ctl;
        long long part_k[prot::kFinalizeBlocks];
        double part_c[prot::kFinalizeBlocks];
        prot::OtInfo ot;
    } *stage = nullptr;              // pinned host memory

    int64_t *rtime = nullptr;        // round timer (PROT_DEBUG_ROUND_TIMES=1)
    int32_t cost_path = PROT_COST_AUTO;    // prot_set_cost_path
    int32_t cost_metric = PROT_METRIC_SQEUCLIDEAN;  // prot_set_cost_metric
    float *l1_buf = nullptr;         // normalised vectors of the L1 image cost
    int64_t l1_cap = 0;
    int loop_groups = 8;             // barrier groups of the phase loop (PROT_LOOP_GROUPS)
    float *mfma_buf = nullptr;       // amax, emax, tile maxima of the matrix-core build
    int64_t mfma_cap = 0;
    int64_t rtime_start = 0;
    double *loss_part = nullptr;     // partial sums of prot_ot_loss_fwd
    int64_t loss_cap = 0;
    int wgs_per_cu = 1;              // PROT_LOOP_WGS_PER_CU (diagnostics)
    int max_grid = 0;                // PROT_LOOP_MAX_GRID: cap on the loop's workgroups (0: none)
    int gate_cap = 0;                // PROT_LOOP_GATE_CAP: workgroups the loop's gate admits (0: all)
    int cooperative = 0;             // PROT_LOOP_COOPERATIVE=1: cooperative launch of the loop
    int64_t barrier_ticks = 0;       // PROT_LOOP_BARRIER_TICKS: bounded barrier wait (0: default)
    int grid_npad = -1;
    int grid_tg = -1;
    int grid_max = 0;
    int t_global = 0;                // PROT_LOOP_T_GLOBAL=1: column duals in global memory always
    int wide_rows = 0;               // PROT_LOOP_WIDE_ROWS=1: 18-bit rows at every size
    uint16_t *tpriv = nullptr;       // per-workgroup column duals beyond LDS
    int64_t tpriv_cap = 0;
    // optimal transport through copies (prot_ot_solve)
    struct Ot {
        int64_t cap_b = 0, cap_a = 0, cap_cb = 0, cap_ca = 0, cap_cells = 0;
        int64_t *s_off = nullptr, *d_off = nullptr;
        int32_t *row_pt = nullptr, *col_pt = nullptr, *cnt = nullptr;
        unsigned long long *ymax = nullptr;
        int32_t *mate_a = nullptr, *mate_b = nullptr, *y_a = nullptr, *y_b = nullptr;
        double *rv = nullptr, *qv = nullptr, *R = nullptr, *Q = nullptr;
        prot::OtInfo *info = nullptr;
        // the copies kept as clusters (prot_ot_solve_clustered)
        int64_t ccap_b = 0, ccap_a = 0, ccap_cells = 0, ccap_mask = 0;
        int2 *cw = nullptr;
        unsigned long long *cmask = nullptr, *cmsum = nullptr;
        uint16_t *cstage = nullptr;
        int32_t *cY = nullptr, *cF = nullptr, *cZ = nullptr, *ctop = nullptr, *cbot = nullptr,
                *cG = nullptr, *cact = nullptr, *cneed = nullptr, *czt = nullptr,
                *cloff = nullptr, *cllen = nullptr;
        uint32_t *csync = nullptr;
        int64_t *cPF = nullptr, *cPG = nullptr;
    } ot;
    // 0 build start, 1 build end, 4 all done (2, 3 unused: the loop's own
    // events are in loop_ev)
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    // start and end of the last kLoopEvents phase-loop launches (a ring;
    // loop_slot is the latest, loop_launches counts them all)
    static constexpr int kLoopEvents = 1024;
    hipEvent_t loop_ev[kLoopEvents][2] = {};
    int loop_slot = -1;
    int64_t loop_launches = 0;
};

namespace {

int fail(prot_ctx *c, int code, const char *fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

int hip_fail(prot_ctx *c, hipError_t e, const char *what)
{
    return fail(c, PROT_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr)                                              \
    do {                                                                \
        hipError_t e_ = (expr);                                         \
        if (e_ != hipSuccess) return hip_fail((ctx), e_, #expr);        \
    } while (0)

// Whether solve_cost / solve_points store the rounded costs as bytes.
int choose_k8(prot_ctx *c, const prot_opts *o, double ei, int *k8)
{
    const int32_t type = o ? o->k_type : PROT_KTYPE_AUTO;
    if (type < PROT_KTYPE_AUTO || type > PROT_KTYPE_UINT8)
        return fail(c, PROT_E_ARG, "unknown k_type %d", (int)type);
    const double K = std::floor(1.0 / ei);
    if (type == PROT_KTYPE_UINT8 && K > 253.0)
        return fail(c, PROT_E_UNSUPPORTED, "a byte matrix needs floor(1/eps) <= 253 (it is %g)", K);
    // AUTO keeps int16: on MI355X the byte matrix halves memory and the cost
    // build's writes, but the scan (latency-bound, with the widening to
    // int16 lanes) runs 10-30% slower.
    *k8 = type == PROT_KTYPE_UINT8;
    return PROT_OK;
}

bool eps_valid(double eps)
{
    return eps > 0.0 && eps < 1.0 && std::floor(1.0 / eps) + 2.0 <= 32767.0;
}

double eps_internal(double eps, const prot_opts *o)
{
    return (o && o->eps_mode == PROT_EPS_STRICT) ? eps / 3.0 : eps;
}

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// Largest k a rounded-cost matrix may hold (int16 entries k <= 32765, so
// that every |y| <= K + 2 fits the loop's 15-bit fields).
constexpr int64_t kKMaxAccepted = 32765;

// The watchdog's phase bound for n_b rows, n_a columns, largest cost K and
// threshold T: Lemma 3.2 keeps every |y| <= K + 2, and Phi = sum y(b) -
// sum y(a) starts at n_b and grows by exactly |B'| > T in every phase
// (Lemma 3.3), so phases <= ((n_b + n_a)(K + 2) - n_b) / (T + 1). (Eq. (4)
// prints n(1 + 2 eps) for the sum of all 2n duals; Lemma 3.2 gives twice
// that, which is the bound used.) opts->phase_bound > 0 replaces it, < 0
// turns the watchdog off.
int64_t phase_bound_for(const prot_opts *o, int64_t n_b, int64_t n_a, int64_t K, int64_t T)
{
    const int64_t given = o ? o->phase_bound : 0;
    if (given > 0) return given;
    if (given < 0) return 0;
    return ((n_b + n_a) * (K + 2) - n_b) / (T + 1);
}

// collect(): the gate admitted too few workgroups, nothing ran; the caller
// enqueues the loop again with a cooperative launch.
constexpr int kRetryCooperative = 1000;

template <class T>
int dev_alloc(prot_ctx *c, T **p, size_t count)
{
    if (*p) {
        (void)hipFree(*p);
        *p = nullptr;
    }
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(c, PROT_E_NOMEM, "hipMalloc of %zu bytes failed: %s", count * sizeof(T),
                    hipGetErrorString(e));
    }
    return PROT_OK;
}

int ensure_loop(prot_ctx *c, int64_t n)
{
    if (n <= c->cap_n && c->key) return PROT_OK;
    const int64_t cap = n < 1024 ? 1024 : n;
    int rc;
    if ((rc = dev_alloc(c, &c->key, (size_t)cap))) return rc;
    if ((rc = dev_alloc(c, &c->t, (size_t)round_up(cap, 8)))) return rc;
    if ((rc = dev_alloc(c, &c->lists, (size_t)cap * 2))) return rc;
    if ((rc = dev_alloc(c, &c->tlists, (size_t)cap * 4 * prot::kMaxGroups))) return rc;
    // list entries carry tags; fresh memory must not hold one by chance
    HIP_TRY(c, prot::launch_fill_u64(c->tlists, cap * 4 * prot::kMaxGroups, 0ull, c->stream));
    c->cap_n = cap;
    return PROT_OK;
}

int ensure_matrix(prot_ctx *c, int64_t n_b, int64_t n_a)
{
    const int64_t need = n_b * prot_pitch(n_a);
    if (need <= c->cap_mat && c->kmat) return PROT_OK;
    int rc = dev_alloc(c, &c->kmat, (size_t)need);
    if (rc) return rc;
    c->cap_mat = need;
    return PROT_OK;
}

int ensure_thresholds(prot_ctx *c, double eps)
{
    const int32_t need = (int32_t)std::floor(1.0 / eps) + 2;
    if (need <= c->cap_th && c->th) return PROT_OK;
    int rc = dev_alloc(c, &c->th, (size_t)need);
    if (rc) return rc;
    c->cap_th = need;
    return PROT_OK;
}

// PROT_COSTS_AUTO: where the costs of a point-set solve live. A matrix that
// fits the 256 MiB Infinity Cache is built and scanned (its reads are cheaper
// than recomputing); a larger one costs more to write than the recomputation
// in the greedy step, so d = 2, 3 computes costs on the fly.
bool auto_on_the_fly(int32_t d, int64_t n_b, int64_t n_a)
{
    return (d == 2 || d == 3) && 2 * n_b * prot_pitch(n_a) > ((int64_t)256 << 20);
}

// rows n (slots), columns n_a. The column duals live in LDS, 2 bytes per
// column (plus ~1 KB of state), while they fit; beyond that (or with
// PROT_LOOP_T_GLOBAL=1) each workgroup keeps its copy in global memory and
// *t_global is set.
int grid_for(prot_ctx *c, int64_t n, int64_t n_a, int *grid, bool *t_global = nullptr)
{
    const int n_pad = (int)round_up(n_a, 8);
    int lds_max = 0;
    HIP_TRY(c, hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock,
                                     c->device));
    const bool tg = (t_global && (c->t_global || c->wide_rows)) ||
                    (int64_t)n_pad * 2 + 2048 > lds_max;
    if (tg && !t_global)
        return fail(c, PROT_E_UNSUPPORTED,
                    "%lld columns: the column duals (2 bytes each) exceed the %d bytes of LDS",
                    (long long)n_a, lds_max);
    if (t_global) *t_global = tg;
    if (c->grid_npad != n_pad || c->grid_tg != (int)tg) {
        int gm = 0;
        hipError_t e = tg ? prot::loop_grid_tg(c->wgs_per_cu, &gm)
                          : prot::loop_grid(n_pad, c->wgs_per_cu, &gm);
        if (e != hipSuccess) return hip_fail(c, e, "occupancy query");
        if (gm <= 0)
            return fail(c, PROT_E_UNSUPPORTED, "%lld columns: the column duals do not fit in LDS",
                        (long long)n_a);
        c->grid_npad = n_pad;
        c->grid_tg = (int)tg;
        c->grid_max = gm;
    }
    const int wpg = prot::kLoopThreads / 64;
    // keys and free lists hold a row in 17 bits, or 18 with duals up to 16,383
    if (n > 262143)
        return fail(c, PROT_E_UNSUPPORTED, "%lld rows: at most 262,143", (long long)n);
    // every wave serves at most 64 rows of B' (one per lane)
    const int64_t min_grid = (n + 64 * wpg - 1) / (64 * wpg);
    if (min_grid > c->grid_max)
        return fail(c, PROT_E_UNSUPPORTED, "n=%lld needs %lld resident workgroups, %d fit",
                    (long long)n, (long long)min_grid, c->grid_max);
    int64_t g = (n + wpg - 1) / wpg;  // one row per wave when n is small
    if (g > c->grid_max) g = c->grid_max;
    if (c->max_grid > 0 && g > c->max_grid) g = std::max<int64_t>(c->max_grid, min_grid);
    if (g < 1) g = 1;
    *grid = (int)g;
    return PROT_OK;
}

// Workspace of the matrix-core build for `batch` instances of at most n_max
// points; leaves j.mfma unset (tiled path) when d is small or it is disabled.
int setup_mfma(prot_ctx *c, prot::PointsJob &j, int64_t n_max, float **buf, int64_t *cap)
{
    j.mfma = prot::MfmaAux{};
    const int32_t from_d = c->cost_path == PROT_COST_MATRIX_CORES ? prot::kMfmaMinD
                           : c->cost_path == PROT_COST_AUTO       ? prot::kMfmaAutoD
                                                                  : INT32_MAX;
    if (j.d < from_d || j.na_single ||
        j.metric != PROT_METRIC_SQEUCLIDEAN || j.k8)
        return PROT_OK;  // (unbalanced instances and other metrics take the direct path)
    const int64_t tx = (n_max + prot::kMfmaTile - 1) / prot::kMfmaTile;
    const int64_t need = 2 * (int64_t)j.batch + (int64_t)j.batch * tx * tx;
    if (need > *cap || !*buf) {
        int rc = dev_alloc(c, buf, (size_t)need);
        if (rc) return rc;
        *cap = need;
    }
    j.mfma.amax = *buf;
    j.mfma.emax = *buf + j.batch;
    j.mfma.tile_max = *buf + 2 * j.batch;
    j.mfma.tiles_x = (int32_t)tx;
    j.mfma.tiles_per_inst = tx * tx;
    j.mfma.cE = prot::mfma_error_constant(j.d);
    return PROT_OK;
}

// Single-instance point build into k (thresholds in the context workspace).
// Workspace of the pruned exact maximum: 16 extreme keys, 12 box bounds, 2
// counts, then two candidate lists of n indices.
int setup_prune(prot_ctx *c, prot::PointsJob &j, int64_t n)  // n: max(rows, columns)
{
    j.prune = prot::PruneAux{};
    j.mpart = nullptr;
    if ((j.d == 2 || j.d == 3) && j.metric != PROT_METRIC_L1_NORMALIZED) {
        const int64_t need = prot::max_parts_cap(n);
        if (need > c->mpart_cap || !c->mpart) {
            int rc = dev_alloc(c, &c->mpart, (size_t)need);
            if (rc) return rc;
            c->mpart_cap = need;
        }
        j.mpart = c->mpart;
    }
    // below this size the plain n^2 pass is cheaper than the four pruning
    // launches (measured: 28 us for n = 10,000, d = 2)
    if ((j.d != 2 && j.d != 3) || n < c->prune_min_n || j.metric == PROT_METRIC_L1_NORMALIZED)
        return PROT_OK;
    if (n > c->prune_cap || !c->prune_buf) {
        int rc = dev_alloc(c, &c->prune_buf, (size_t)(256 + 8 * std::max<int64_t>(n, 1024)));
        if (rc) return rc;
        c->prune_cap = std::max<int64_t>(n, 1024);
    }
    j.prune.ext = reinterpret_cast<unsigned long long *>(c->prune_buf);
    j.prune.bb = reinterpret_cast<uint32_t *>(c->prune_buf + 128);
    j.prune.cnt = reinterpret_cast<uint32_t *>(c->prune_buf + 192);
    j.prune.cx = reinterpret_cast<int32_t *>(c->prune_buf + 256);
    j.prune.cy = j.prune.cx + c->prune_cap;
    return PROT_OK;
}

prot::PointsJob points_job(prot_ctx *c, const float *X, const float *Y, int64_t n, int32_t d,
                           double eps, int16_t *k, int64_t ldk, int64_t n_a = 0)
{
    prot::PointsJob j{};
    j.X = X;
    j.Y = Y;
    j.n_single = n;
    j.na_single = (n_a && n_a != n) ? n_a : 0;
    j.ldk_single = ldk;
    j.d = d;
    j.batch = 1;
    j.eps = eps;
    j.k = k;
    j.m = &c->ctl->m;
    j.th = c->th;
    j.kcap = (int32_t)std::floor(1.0 / eps) + 2;
    j.err = &c->ctl->err;
    j.kmax_out = &c->ctl->kmax;
    j.metric = c->cost_metric;
    return j;
}

// The L1 image cost normalises X and Y into a workspace first.
int setup_l1(prot_ctx *c, prot::PointsJob &j, int64_t n_b, int64_t n_a)
{
    if (j.metric != PROT_METRIC_L1_NORMALIZED) return PROT_OK;
    if (j.d > 12288)
        return fail(c, PROT_E_UNSUPPORTED, "the L1 image cost takes d <= 12288 (d = %d)", j.d);
    const int64_t need = (n_b + n_a) * (int64_t)j.d;
    if (need > c->l1_cap || !c->l1_buf) {
        int rc = dev_alloc(c, &c->l1_buf, (size_t)need);
        if (rc) return rc;
        c->l1_cap = need;
    }
    j.l1_x = c->l1_buf;
    j.l1_y = c->l1_buf + n_b * (int64_t)j.d;
    return PROT_OK;
}

// finalize/collect cost kind of a point-set solve
int points_cost_kind(const prot_ctx *c)
{
    return c->cost_metric == PROT_METRIC_EUCLIDEAN        ? 3
           : c->cost_metric == PROT_METRIC_L1_NORMALIZED ? 4
                                                          : 2;
}

prot::LoopArgs loop_args(prot_ctx *c, const int16_t *k, int64_t n, int64_t n_a, int64_t ldk,
                         int64_t T, const prot_opts *o, int32_t *y_b, int64_t K)
{
    prot::LoopArgs a{};
    a.phase_bound = phase_bound_for(o, n, n_a, K, T);
    a.barrier_ticks = c->barrier_ticks;
    a.k = k;
    a.ldk = ldk;
    a.n = (int32_t)n;
    a.n_a = (int32_t)n_a;
    a.n_pad = (int32_t)round_up(n_a, 8);
    a.T = T;
    a.origin = (o && o->origin_mode == PROT_ORIGIN_ZERO) ? 1 : 0;
    a.max_phases = o ? o->max_phases : 0;
    a.key = c->key;
    a.t = c->t;
    a.y_b = y_b;
    const int64_t region = c->cap_n * prot::kMaxGroups;
    a.F[0] = c->tlists;
    a.F[1] = c->tlists + region;
    a.L[0] = c->tlists + 2 * region;
    a.L[1] = c->tlists + 3 * region;
    a.list_cap = c->cap_n;
    a.words = c->words;
    a.ctl = c->ctl;
    a.trace = c->trace;
    a.rtime = c->rtime;
    return a;
}

// Enqueue init, the phase loop and the completion; returns after enqueueing.
// Costs computed on the fly from points of dimension d (d = 0: read k).
struct OnTheFly {
    int32_t d = 0;
    const float *X = nullptr, *Y = nullptr;
    double eps = 0.0;
    uint32_t switch_round = 0;  // hand over to the stored matrix (LoopArgs)
};

// Copies of the transport reduction: row b reads cost row rmap[b]; ymax holds
// the largest dual of each point's copies.
struct Copies {
    const int32_t *rmap = nullptr;
    unsigned long long *ymax = nullptr;
};

// The events of the next phase-loop launch: the ring's next slot (its
// events created on first use).
int next_loop_events(prot_ctx *c, hipEvent_t **out)
{
    const int slot = (c->loop_slot + 1) % prot_ctx::kLoopEvents;
    for (hipEvent_t &e : c->loop_ev[slot])
        if (!e && hipEventCreate(&e) != hipSuccess)
            return fail(c, PROT_E_HIP, "event creation failed");
    c->loop_slot = slot;
    c->loop_launches += 1;
    *out = c->loop_ev[slot];
    return PROT_OK;
}

// The phase loop on n rows (B) and n_a >= n columns (A), with its init and
// finish kernels. K: the largest rounded cost (for the watchdog and the
// warm-start check). cooperative: launch the loop cooperatively (the retry after the gate
// admitted too few workgroups).
int run_loop(prot_ctx *c, const int16_t *k, int64_t n, int64_t n_a, int64_t ldk, int64_t T,
             const prot_opts *o, int32_t warm, int32_t *mate_a, int32_t *mate_b, int32_t *y_a,
             int32_t *y_b, int64_t K, bool cooperative = false,
             const OnTheFly &otf = OnTheFly(), const Copies &cp = Copies(), int k8 = 0,
             int64_t trace_off = 0)
{
    int rc = ensure_loop(c, n_a);
    if (rc) return rc;
    int grid = 0;
    bool tg = false;
    if ((rc = grid_for(c, n, n_a, &grid, &tg))) return rc;
    // more than 131,071 rows travel in 18 bits, their duals in 14 (a matrix
    // given as rounded costs has no known K: a dual that outgrows 14 bits
    // then stops the loop with PROT_E_STATE)
    const bool wide = n > 131071 || c->wide_rows;  // n_a >= n: then tg holds too
    if (wide && K + 2 > 0x3FFF && K < kKMaxAccepted)
        return fail(c, PROT_E_UNSUPPORTED,
                    "%lld rows: above 131,071 rows the duals must stay below 16,384 "
                    "(largest rounded cost %lld; eps >= 1/16381)",
                    (long long)n, (long long)K);
    if (tg) {
        const int64_t need = (int64_t)grid * round_up(n_a, 8);
        if (need > c->tpriv_cap) {
            if ((rc = dev_alloc(c, &c->tpriv, (size_t)need))) return rc;
            c->tpriv_cap = need;
        }
    }
    prot::LoopArgs a = loop_args(c, k, n, n_a, ldk, T, o, y_b, K);
    a.wide = wide ? 1 : 0;
    a.tpriv = tg ? c->tpriv : nullptr;
    a.groups = std::min(c->loop_groups, grid);
    a.gated = (c->cooperative || cooperative) ? 0 : 1;
    a.gate_cap = c->gate_cap;
    a.rmap = cp.rmap;
    a.ymax = cp.ymax;
    a.k8 = k8;
    if (otf.d) {
        a.pd = otf.d;
        a.px = otf.X;
        a.py = otf.Y;
        a.pm = &c->ctl->m;
        a.pth = c->th;
        a.peps = otf.eps;
        a.switch_round = otf.switch_round;
    }
    // a continuation records its phases after those of the launch before
    // (when the watchdog bounds them within the trace)
    if (trace_off > 0)
        a.trace = a.phase_bound > 0 && trace_off + a.phase_bound <= prot::kTraceCap
                      ? c->trace + 4 * trace_off
                      : nullptr;
    if (warm) {
        // (I1), Lemma 3.2's bound on the duals and the matching structure of
        // the given state, O(n); on request (I2), O(n_b n_a).
        HIP_TRY(c, prot::launch_clear_err(c->ctl, c->stream));
        HIP_TRY(c, prot::launch_check_state(n, n_a, mate_a, mate_b, y_a, y_b,
                                            (int32_t)std::min<int64_t>(K + 2, wide ? 0x3FFF : 0x7FFF),
                                            c->ctl, c->stream));
        const bool i2 = o && o->check_warm && k && !k8 && !otf.d;
        if (i2)
            HIP_TRY(c, prot::launch_check_feasible(k, ldk, n, n_a, mate_b, y_a, y_b, c->ctl,
                                                   c->stream));
        HIP_TRY(c, hipMemcpyAsync(&c->stage->ctl.err, &c->ctl->err, sizeof(int32_t),
                                  hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        if (c->stage->ctl.err & 2)
            return fail(c, PROT_E_STATE,
                        i2 ? "warm-start state is not a matching satisfying (I1) and (I2) "
                             "with |y| <= K + 2"
                           : "warm-start state is not a matching satisfying (I1) with "
                             "|y| <= K + 2");
    }
    // a relaunch after the gate admitted too few workgroups: that attempt ran
    // nothing, only its error bit goes
    if (cooperative) HIP_TRY(c, prot::launch_clear_err(c->ctl, c->stream, 16));
    HIP_TRY(c, prot::launch_init(a, warm, mate_a, mate_b, y_a, c->stream));
    if (c->rtime) HIP_TRY(c, prot::launch_clear_times(c->rtime, c->stream));
    hipEvent_t *le = nullptr;
    if (int r = next_loop_events(c, &le)) return r;
    HIP_TRY(c, prot::launch_loop(a, grid, c->stream, le[0], le[1]));
    const int32_t complete = (o && o->no_completion) ? 0 : 1;
    HIP_TRY(c, prot::launch_finish(a, warm, complete, mate_a, mate_b, y_a, c->lists, c->stream));
    return PROT_OK;
}

// Status of a loop from its control block (host copy): an error code, or
// PROT_OK / PROT_PARTIAL / PROT_E_PHASE_BOUND.
int loop_status(prot_ctx *c, const Ctl &h)
{
    if (h.err & 4) return fail(c, PROT_E_HIP, "phase loop: a list entry was not published in time");
    if (h.err & 32) return fail(c, PROT_E_HIP, "phase loop: a round barrier timed out");
    if (h.err & 8) return fail(c, PROT_E_UNSUPPORTED, "phase loop: more than 2^32 rounds");
    if (h.err & 64)
        return fail(c, PROT_E_STATE, "phase loop: a dual left the range of Lemma 3.2 (the "
                                     "warm start is not a state the method reaches)");
    if (h.err & 16)
        return fail(c, PROT_E_HIP, "phase loop: too few workgroups resident for the rows "
                                   "(the GPU is busy; nothing ran)");
    if (h.status == 2)
        return fail(c, PROT_E_PHASE_BOUND,
                    "phase loop: stopped by the phase-bound watchdog after %lld phases (the "
                    "outputs hold the state reached)",
                    (long long)h.phases);
    return h.status ? PROT_PARTIAL : PROT_OK;
}

int collect(prot_ctx *c, prot_stats *st, int64_t T, double eps_int, int cost_kind,
            bool timed_build, bool may_retry = false)
{
    static_assert(offsetof(prot_ctx::Stage, part_k) == offsetof(Report, part_k) &&
                      offsetof(prot_ctx::Stage, part_c) == offsetof(Report, part_c),
                  "the host stage begins with the device report's layout");
    HIP_TRY(c, hipMemcpyAsync(c->stage, c->rep, sizeof(Report), hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const Ctl &h = c->stage->ctl;
    // nothing ran: the state is as it was given, so the loop can run again
    if ((h.err & 16) && !(h.err & prot::kErrLoop) && may_retry && !c->cooperative)
        return kRetryCooperative;
    const int ls = loop_status(c, h);
    if (ls < 0 && ls != PROT_E_PHASE_BOUND) return ls;
    if (!st) return ls;
    std::memset(st, 0, sizeof(*st));
    st->phases = h.phases;
    st->sum_free = h.sum_free;
    st->rounds = h.rounds;
    st->max_rounds = h.max_rounds;
    st->scanned = (int64_t)h.scanned;
    st->threshold = T;
    st->status = ls;
    st->eps_internal = eps_int;
    long long sk = 0;
    double sc = 0.0;
    for (int i = 0; i < prot::kFinalizeBlocks; ++i) {
        sk += c->stage->part_k[i];
        sc += c->stage->part_c[i];
    }
    st->sum_k = sk;
    st->cost_scale = 1.0;
    if (cost_kind == 1) st->cost = sc;
    if (cost_kind == 2) {
        st->cost_scale = (double)h.m;
        st->cost = h.m > 0.0f ? sc / (double)h.m : 0.0;
    }
    if (cost_kind == 3) {  // Euclidean: c = sqrt(d2 / m)
        st->cost_scale = (double)h.m;
        st->cost = h.m > 0.0f ? sc / std::sqrt((double)h.m) : 0.0;
    }
    if (cost_kind == 4) {  // L1 of normalised vectors, halved
        st->cost_scale = 2.0;
        st->cost = sc;
    }
    st->kmax = h.kmax;
    float ms = 0.0f;
    if (timed_build && hipEventElapsedTime(&ms, c->ev[0], c->ev[1]) == hipSuccess)
        st->ms_build = ms;
    if (c->loop_slot >= 0 &&
        hipEventElapsedTime(&ms, c->loop_ev[c->loop_slot][0], c->loop_ev[c->loop_slot][1]) ==
            hipSuccess)
        st->ms_loop_kernel = ms;
    if (hipEventElapsedTime(&ms, c->ev[timed_build ? 0 : 1], c->ev[4]) == hipSuccess)
        st->ms_total = ms;
    return PROT_OK;
}

void fill_match_counts(prot_ctx *c, int64_t n, prot_stats *st, const prot_opts *o)
{
    if (!st) return;
    const int64_t free_after = c->stage->ctl.free_after;
    st->matched_in_phases = n - free_after;
    st->completed_pairs =
        ((o && o->no_completion) || st->status != PROT_OK) ? 0 : free_after;
}

// |B| = 0 with |A| > 0: nothing to match; a cold start still hands back the
// initial column state (every a free, y(a) = 0).
int no_rows(prot_ctx *c, int64_t n_a, int32_t warm, int32_t *mate_a, int32_t *y_a)
{
    if (warm || n_a <= 0) return PROT_OK;
    if (!mate_a || !y_a) return fail(c, PROT_E_ARG, "null column output");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipMemsetAsync(mate_a, 0xFF, sizeof(int32_t) * n_a, c->stream));
    HIP_TRY(c, hipMemsetAsync(y_a, 0, sizeof(int32_t) * n_a, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return PROT_OK;
}

}  // namespace

struct prot_batch {
    prot_ctx *ctx = nullptr;
    int32_t batch = 0, d = 0, n_max = 0;
    int64_t ldk_max = 0;
    double eps = 0.0;
    prot_opts opts{};
    int grid = 1;
    int32_t *order = nullptr, *n_arr = nullptr, *ldk_arr = nullptr;
    int64_t *pt_off = nullptr, *k_off = nullptr;
    int16_t *k = nullptr;
    float *m = nullptr, *th = nullptr;
    int32_t kcap = 0;
    int32_t *err = nullptr;
    unsigned int *queue = nullptr;
    prot_instance_stats *stats_tmp = nullptr;
    float *mfma_buf = nullptr;
    int64_t mfma_cap = 0;
    prot::MfmaAux mfma{};
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // Teams (instances above the LDS-resident limit of 1024): `team`
    // phase-loop workgroups per instance, per_launch instances per launch.
    int team = 0;
    int per_launch = 0;
    int32_t n_pad_max = 0;
    prot::LoopArgs *loops = nullptr;
    unsigned long long *t_key = nullptr, *t_lists = nullptr, *t_words = nullptr;
    uint16_t *t_t = nullptr;
    uint32_t *t_skip = nullptr;
    Ctl *t_ctl = nullptr;
    int32_t *t_scratch = nullptr;
    double *loss_part = nullptr;     // partial sums of the loss forward
};

namespace {

template <class T>
int upload(prot_ctx *c, T **dst, const std::vector<T> &src)
{
    int rc = dev_alloc(c, dst, src.size());
    if (rc) return rc;
    HIP_TRY(c, hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return PROT_OK;
}

// Chooses between the LDS-resident batched kernel (instances up to n = 1024)
// and teams of phase-loop workgroups (larger instances), and for teams builds
// every instance's loop arguments and workspace. PROT_BATCH_TEAM=<w> forces
// w workgroups per instance (0: never use teams).
int setup_teams(prot_ctx *c, prot_batch *bp, const std::vector<int32_t> &n_arr,
                const std::vector<int32_t> &ldk, const std::vector<int64_t> &pt_off,
                const std::vector<int64_t> &k_off, const prot_batch_config *cfg)
{
    int forced = -1;  // -1 automatic, 0 LDS engine, > 0 that team size
    if (cfg && cfg->engine == PROT_BATCH_ENGINE_LDS) forced = 0;
    else if (cfg && cfg->engine == PROT_BATCH_ENGINE_TEAMS) forced = cfg->team > 0 ? cfg->team : -2;
    else if (const char *v = std::getenv("PROT_BATCH_TEAM")) forced = std::atoi(v);
    const bool must = cfg && cfg->engine == PROT_BATCH_ENGINE_TEAMS;
    if (forced == 0 || (forced == -1 && bp->n_max <= 1024)) return PROT_OK;
    const int32_t n_pad_max = (int32_t)round_up(bp->n_max, 8);
    int gm = 0;
    hipError_t e = prot::loop_grid_multi(n_pad_max, c->wgs_per_cu, &gm);
    if (e != hipSuccess) return hip_fail(c, e, "team occupancy");
    if (gm < 1) return PROT_OK;  // keep the LDS-resident kernel
    // each wave serves at most 64 rows of B' (one per lane): a team needs
    // ceil(n_max / (64 * 16)) workgroups at least
    const int wpg = prot::kLoopThreads / 64;
    const int team_min = (int)((bp->n_max + 64 * wpg - 1) / (64 * wpg));
    if (must && (forced > 8 || (forced > 0 && forced < team_min)))
        return fail(c, PROT_E_UNSUPPORTED, "team of %d workgroups for n_max = %d", forced,
                    (int)bp->n_max);
    int team = forced > 0 ? forced : gm / bp->batch;
    team = std::max(team_min, std::min(team, 8));
    if (team > gm) {
        if (must) return fail(c, PROT_E_UNSUPPORTED, "a team of %d does not fit", team);
        return PROT_OK;  // keep the LDS-resident kernel
    }
    bp->team = team;
    bp->per_launch = gm / team;
    bp->n_pad_max = n_pad_max;
    const int32_t batch = bp->batch;
    const int G = std::min(team, 8);
    int64_t nk = 0, nt = 0, nl = 0, ns = 0;
    for (int32_t i = 0; i < batch; ++i) {
        nk += n_arr[i];
        nt += round_up(n_arr[i], 8);
        nl += (int64_t)4 * G * n_arr[i];
        ns += 2 * (int64_t)n_arr[i];
    }
    const int64_t words_per = (int64_t)3 * prot::kMaxGroups * prot::kWordStride;
    int rc = dev_alloc(c, &bp->t_key, (size_t)nk);
    if (!rc) rc = dev_alloc(c, &bp->t_t, (size_t)nt);
    if (!rc) rc = dev_alloc(c, &bp->t_lists, (size_t)nl);
    if (!rc) rc = dev_alloc(c, &bp->t_words, (size_t)(words_per * batch));
    if (!rc) rc = dev_alloc(c, &bp->t_ctl, (size_t)batch);
    if (!rc) rc = dev_alloc(c, &bp->t_scratch, (size_t)ns);
    if (!rc) rc = dev_alloc(c, &bp->t_skip, (size_t)nk);
    if (rc) return rc;
    // list entries carry tags, so fresh memory must hold none by chance
    HIP_TRY(c, hipMemset(bp->t_lists, 0, sizeof(unsigned long long) * (size_t)nl));
    HIP_TRY(c, hipMemset(bp->t_ctl, 0, sizeof(Ctl) * (size_t)batch));
    std::vector<prot::LoopArgs> la(batch);
    const int origin = bp->opts.origin_mode == PROT_ORIGIN_ZERO ? 1 : 0;
    int64_t ok = 0, ot = 0, ol = 0;
    for (int32_t i = 0; i < batch; ++i) {
        prot::LoopArgs &a = la[i];
        const int64_t n = n_arr[i];
        a.k = bp->k + k_off[i];
        a.ldk = ldk[i];
        a.n = (int32_t)n;
        a.n_a = (int32_t)n;
        a.n_pad = (int32_t)round_up(n, 8);
        a.T = prot_threshold(bp->eps, n);
        a.origin = origin;
        a.max_phases = bp->opts.max_phases;
        a.phase_bound = phase_bound_for(&bp->opts, n, n, (int64_t)std::floor(1.0 / bp->eps), a.T);
        a.key = bp->t_key + ok;
        a.skip = bp->t_skip + ok;
        a.t = bp->t_t + ot;
        a.y_b = nullptr;  // the launch's y_b base + y_off
        for (int q = 0; q < 2; ++q) {
            a.F[q] = bp->t_lists + ol + (int64_t)q * G * n;
            a.L[q] = bp->t_lists + ol + (int64_t)(2 + q) * G * n;
        }
        a.list_cap = n;
        a.groups = G;
        a.words = bp->t_words + words_per * i;
        a.ctl = bp->t_ctl + i;
        a.trace = nullptr;
        a.rtime = nullptr;
        a.y_off = pt_off[i];
        ok += n;
        ot += round_up(n, 8);
        ol += (int64_t)4 * G * n;
    }
    return upload(c, &bp->loops, la);
}

int batch_enqueue(prot_batch *bp, hipStream_t s, const float *X, const float *Y, int32_t *mate_a,
                  int32_t *mate_b, int32_t *y_a, int32_t *y_b, prot_instance_stats *stats)
{
    prot_ctx *c = bp->ctx;
    prot::PointsJob j{};
    j.X = X;
    j.Y = Y;
    j.pt_off = bp->pt_off;
    j.n_arr = bp->n_arr;
    j.k_off = bp->k_off;
    j.ldk_arr = bp->ldk_arr;
    j.d = bp->d;
    j.batch = bp->batch;
    j.eps = bp->eps;
    j.k = bp->k;
    j.m = bp->m;
    j.th = bp->th;
    j.kcap = bp->kcap;
    j.err = bp->err;
    j.mfma = bp->mfma;
    HIP_TRY(c, prot::launch_points(j, bp->n_max, bp->ldk_max, s));
    if (bp->team > 0) {
        prot::TeamArgs t{};
        t.batch = bp->batch;
        t.d = bp->d;
        t.complete = bp->opts.no_completion ? 0 : 1;
        t.eps = bp->eps;
        t.loops = bp->loops;
        t.pt_off = bp->pt_off;
        t.X = X;
        t.Y = Y;
        t.m = bp->m;
        t.mate_a = mate_a;
        t.mate_b = mate_b;
        t.y_a = y_a;
        t.y_b = y_b;
        t.scratch = bp->t_scratch;
        t.stats = reinterpret_cast<prot::InstanceStats *>(stats ? stats : bp->stats_tmp);
        t.err = bp->err;
        HIP_TRY(c, prot::launch_team_init(t, bp->n_pad_max, s));
        for (int first = 0; first < bp->batch; first += bp->per_launch) {
            const int count = std::min(bp->per_launch, bp->batch - first);
            HIP_TRY(c, prot::launch_loop_multi(bp->loops + first, count, bp->team, bp->n_pad_max,
                                               y_b, s));
        }
        HIP_TRY(c, prot::launch_team_finish(t, s));
        return PROT_OK;
    }
    prot::BatchArgs a{};
    a.batch = bp->batch;
    a.d = bp->d;
    a.eps = bp->eps;
    a.max_phases = bp->opts.max_phases;
    a.origin = bp->opts.origin_mode == PROT_ORIGIN_ZERO ? 1 : 0;
    a.complete = bp->opts.no_completion ? 0 : 1;
    a.order = bp->order;
    a.n_arr = bp->n_arr;
    a.ldk_arr = bp->ldk_arr;
    a.pt_off = bp->pt_off;
    a.k_off = bp->k_off;
    a.k = bp->k;
    a.X = X;
    a.Y = Y;
    a.m = bp->m;
    a.mate_a = mate_a;
    a.mate_b = mate_b;
    a.y_a = y_a;
    a.y_b = y_b;
    a.stats = reinterpret_cast<prot::InstanceStats *>(stats ? stats : bp->stats_tmp);
    a.queue = bp->queue;
    a.rtime = c->rtime;
    a.err = bp->err;
    HIP_TRY(c, prot::launch_batch_solve(a, bp->n_max, bp->grid, s));
    return PROT_OK;
}

// Status of a batch from its error word: bit 0 a non-finite coordinate,
// bits 2, 3, 5, 6 a failed loop of some instance, bit 8 an instance stopped
// by the phase-bound watchdog.
int batch_err_status(prot_ctx *c, int32_t err)
{
    if (err & 1) return fail(c, PROT_E_RANGE, "a point coordinate is not finite");
    if (err & (4 | 32))
        return fail(c, PROT_E_HIP, "phase loop: a list entry or a round barrier timed out");
    if (err & 8) return fail(c, PROT_E_UNSUPPORTED, "phase loop: more than 2^32 rounds");
    if (err & 64) return fail(c, PROT_E_STATE, "phase loop: a dual left the range of Lemma 3.2");
    if (err & 256)
        return fail(c, PROT_E_PHASE_BOUND, "an instance was stopped by the phase-bound watchdog");
    return PROT_OK;
}

bool batch_args_ok(const prot_batch *bp, const float *X, const float *Y, const int32_t *mate_a,
                   const int32_t *mate_b, const int32_t *y_a, const int32_t *y_b)
{
    return bp && X && Y && mate_a && mate_b && y_a && y_b;
}

}  // namespace

static_assert(sizeof(prot_instance_stats) == sizeof(prot::InstanceStats),
              "prot_instance_stats and InstanceStats must match");

extern "C" {

int64_t prot_pitch(int64_t n) { return n <= 0 ? 128 : round_up(n, 128); }

int64_t prot_threshold(double eps, int64_t n) { return (int64_t)std::floor(eps * (double)n + 1e-9); }

const char *prot_status_string(int s)
{
    switch (s) {
    case PROT_OK: return "ok";
    case PROT_PARTIAL: return "partial (max_phases reached)";
    case PROT_E_ARG: return "invalid argument";
    case PROT_E_RANGE: return "cost out of range or not finite";
    case PROT_E_EPS: return "eps out of range";
    case PROT_E_PHASE_BOUND: return "stopped by the phase-bound watchdog";
    case PROT_E_STATE: return "invalid warm-start state";
    case PROT_E_HIP: return "HIP runtime error";
    case PROT_E_NOMEM: return "out of device memory";
    case PROT_E_UNSUPPORTED: return "unsupported size";
    default: return "unknown status";
    }
}

// Message of the last failed call that takes no context, on this thread.
static thread_local std::string g_free_err;

const char *prot_last_error(prot_ctx *ctx)
{
    if (ctx) return ctx->err.c_str();
    return g_free_err.empty() ? "null context" : g_free_err.c_str();
}

int prot_ctx_create(prot_ctx **out, int device, void *hip_stream)
{
    if (!out) return PROT_E_ARG;
    *out = nullptr;
    prot_ctx *c = new (std::nothrow) prot_ctx();
    if (!c) return PROT_E_NOMEM;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) {
        delete c;
        return PROT_E_HIP;
    }
    int rc = dev_alloc(c, &c->rep, 1);
    if (!rc && hipMemset(c->rep, 0, sizeof(Report)) != hipSuccess) rc = PROT_E_HIP;
    if (!rc) {
        c->ctl = &c->rep->ctl;
        c->part_k = c->rep->part_k;
        c->part_c = c->rep->part_c;
    }
    if (!rc) rc = dev_alloc(c, &c->words, (size_t)3 * prot::kMaxGroups * prot::kWordStride);
    if (!rc) rc = dev_alloc(c, &c->trace, (size_t)4 * prot::kTraceCap);
    if (!rc && hipHostMalloc((void **)&c->stage, sizeof(prot_ctx::Stage), hipHostMallocDefault) !=
                   hipSuccess)
        rc = PROT_E_NOMEM;
    for (int i = 0; i < 5 && !rc; ++i)
        if (hipEventCreate(&c->ev[i]) != hipSuccess) rc = PROT_E_HIP;
    if (const char *v = std::getenv("PROT_COST_PATH"))
        c->cost_path = std::strcmp(v, "mfma") == 0     ? PROT_COST_MATRIX_CORES
                       : std::strcmp(v, "direct") == 0 ? PROT_COST_DIRECT
                                                       : PROT_COST_AUTO;
    if (const char *v = std::getenv("PROT_PRUNE_MIN_N")) c->prune_min_n = std::atoll(v);
    if (const char *v = std::getenv("PROT_LOOP_GATE_CAP")) c->gate_cap = std::max(0, std::atoi(v));
    if (const char *v = std::getenv("PROT_LOOP_COOPERATIVE")) c->cooperative = std::atoi(v) == 1;
    if (const char *v = std::getenv("PROT_LOOP_BARRIER_TICKS"))
        c->barrier_ticks = std::max<int64_t>(0, std::atoll(v));
    if (const char *v = std::getenv("PROT_LOOP_GROUPS")) {
        const int g = std::atoi(v);
        if (g >= 1 && g <= prot::kMaxGroups) c->loop_groups = g;
    }
    if (const char *v = std::getenv("PROT_LOOP_WGS_PER_CU")) {
        const int w = std::atoi(v);
        if (w >= 1 && w <= 8) c->wgs_per_cu = w;
    }
    if (const char *v = std::getenv("PROT_LOOP_MAX_GRID")) c->max_grid = std::atoi(v);
    if (const char *v = std::getenv("PROT_LOOP_T_GLOBAL")) c->t_global = std::atoi(v) == 1;
    // 18-bit rows at every size (with the column duals in global memory)
    if (const char *v = std::getenv("PROT_LOOP_WIDE_ROWS")) c->wide_rows = std::atoi(v) == 1;
    if (!rc) {
        const char *v = std::getenv("PROT_DEBUG_ROUND_TIMES");
        if (v && v[0] == '1') rc = dev_alloc(c, &c->rtime, (size_t)3 * prot::kRoundTimeCap);
    }
    if (rc) {
        prot_ctx_destroy(c);
        return rc;
    }
    *out = c;
    return PROT_OK;
}

int prot_ctx_destroy(prot_ctx *c)
{
    if (!c) return PROT_E_ARG;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    (void)hipFree(c->key);
    (void)hipFree(c->t);
    (void)hipFree(c->lists);
    (void)hipFree(c->tlists);
    (void)hipFree(c->prune_buf);
    (void)hipFree(c->mpart);
    (void)hipFree(c->words);
    (void)hipFree(c->rep);
    (void)hipFree(c->trace);
    (void)hipFree(c->kmat);
    (void)hipFree(c->tpriv);
    (void)hipFree(c->th);
    (void)hipFree(c->rtime);
    (void)hipFree(c->mfma_buf);
    (void)hipFree(c->l1_buf);
    (void)hipFree(c->loss_part);
    for (void *p : {(void *)c->ot.s_off, (void *)c->ot.d_off, (void *)c->ot.row_pt,
                    (void *)c->ot.col_pt, (void *)c->ot.ymax, (void *)c->ot.cnt,
                    (void *)c->ot.mate_a, (void *)c->ot.mate_b, (void *)c->ot.y_a,
                    (void *)c->ot.y_b, (void *)c->ot.rv, (void *)c->ot.qv, (void *)c->ot.R,
                    (void *)c->ot.Q, (void *)c->ot.info, (void *)c->ot.cw, (void *)c->ot.cmask, (void *)c->ot.cmsum,
                    (void *)c->ot.cstage, (void *)c->ot.cact, (void *)c->ot.cneed,
                    (void *)c->ot.czt, (void *)c->ot.cloff, (void *)c->ot.cllen,
                    (void *)c->ot.csync, (void *)c->ot.cY, (void *)c->ot.cF, (void *)c->ot.cZ,
                    (void *)c->ot.ctop, (void *)c->ot.cbot, (void *)c->ot.cG, (void *)c->ot.cPF,
                    (void *)c->ot.cPG})
        (void)hipFree(p);
    if (c->stage) (void)hipHostFree(c->stage);
    for (int i = 0; i < 5; ++i)
        if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
    for (auto &pair : c->loop_ev)
        for (hipEvent_t e : pair)
            if (e) (void)hipEventDestroy(e);
    delete c;
    return PROT_OK;
}

int prot_set_cost_metric(prot_ctx *c, int32_t metric)
{
    if (!c) return PROT_E_ARG;
    if (metric != PROT_METRIC_SQEUCLIDEAN && metric != PROT_METRIC_EUCLIDEAN &&
        metric != PROT_METRIC_L1_NORMALIZED)
        return fail(c, PROT_E_ARG, "unknown cost metric %d", (int)metric);
    c->cost_metric = metric;
    return PROT_OK;
}

int prot_set_cost_path(prot_ctx *c, int32_t path)
{
    if (!c) return PROT_E_ARG;
    if (path != PROT_COST_DIRECT && path != PROT_COST_MATRIX_CORES && path != PROT_COST_AUTO)
        return fail(c, PROT_E_ARG, "unknown cost path %d", (int)path);
    c->cost_path = path;
    return PROT_OK;
}

int prot_set_stream(prot_ctx *c, void *hip_stream)
{
    if (!c) return PROT_E_ARG;
    c->stream = (hipStream_t)hip_stream;
    return PROT_OK;
}

int prot_reserve(prot_ctx *c, int64_t n_max, int32_t with_matrix)
{
    if (!c || n_max < 0) return fail(c, PROT_E_ARG, "prot_reserve: bad arguments");
    HIP_TRY(c, hipSetDevice(c->device));
    int rc = ensure_loop(c, n_max);
    if (!rc && with_matrix) rc = ensure_matrix(c, n_max, n_max);
    if (!rc) {
        int grid = 0;
        rc = grid_for(c, n_max, n_max, &grid);
    }
    return rc;
}

int64_t prot_max_n(prot_ctx *c)
{
    if (!c) return 0;
    // LDS holds 2 bytes per column; each wave serves at most 64 rows.
    int64_t best = 0;
    for (int64_t n = 4096; n <= (1 << 20); n += 4096) {
        const int n_pad = (int)round_up(n, 8);
        int gm = 0;
        if (prot::loop_grid(n_pad, c->wgs_per_cu, &gm) != hipSuccess || gm <= 0) break;
        if ((n + 64 * 8 - 1) / (64 * 8) > gm) break;
        best = n;
    }
    return best;
}

int prot_round_costs_rect(prot_ctx *c, const float *C, int64_t n_b, int64_t n_a, int64_t ldc,
                          double eps, int16_t *k, int64_t ldk)
{
    if (!c) return PROT_E_ARG;
    if (!C || !k || n_b < 0 || n_a < 0 || ldc < n_a || ldk < n_a || ldk % 8 ||
        ((uintptr_t)k & 15))
        return fail(c, PROT_E_ARG, "prot_round_costs: bad pointer, size or alignment");
    if (!eps_valid(eps)) return fail(c, PROT_E_EPS, "eps=%g not in (0,1) or too small", eps);
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, prot::launch_round_costs(C, n_b, n_a, ldc, eps, k, ldk, c->ctl, c->stream));
    HIP_TRY(c, hipMemcpyAsync(&c->stage->ctl.err, &c->ctl->err, sizeof(int32_t),
                              hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (c->stage->ctl.err & 1) return fail(c, PROT_E_RANGE, "a cost is NaN or outside [0,1]");
    return PROT_OK;
}

int prot_round_costs(prot_ctx *c, const float *C, int64_t n, int64_t ldc, double eps,
                     int16_t *k, int64_t ldk)
{
    return prot_round_costs_rect(c, C, n, n, ldc, eps, k, ldk);
}

int prot_build_costs_rect(prot_ctx *c, const float *X, int64_t n_b, const float *Y, int64_t n_a,
                          int32_t d, double eps, int16_t *k, int64_t ldk, float *m_out)
{
    if (!c) return PROT_E_ARG;
    if (!X || !Y || !k || n_b < 0 || n_a < 0 || d < 1 || ldk < n_a || ldk % 8 ||
        ((uintptr_t)k & 15))
        return fail(c, PROT_E_ARG, "prot_build_costs: bad pointer, size or alignment");
    if (!eps_valid(eps)) return fail(c, PROT_E_EPS, "eps=%g not in (0,1) or too small", eps);
    HIP_TRY(c, hipSetDevice(c->device));
    int rc = ensure_thresholds(c, eps);
    if (rc) return rc;
    const int64_t n_max = std::max(n_b, n_a);
    prot::PointsJob j = points_job(c, X, Y, n_b, d, eps, k, ldk, n_a);
    if ((rc = setup_mfma(c, j, n_max, &c->mfma_buf, &c->mfma_cap))) return rc;
    if ((rc = setup_prune(c, j, n_max))) return rc;
    if ((rc = setup_l1(c, j, n_b, n_a))) return rc;
    HIP_TRY(c, prot::launch_points(j, n_max, ldk, c->stream));
    if (m_out)
        HIP_TRY(c, hipMemcpyAsync(m_out, &c->ctl->m, sizeof(float), hipMemcpyDeviceToDevice,
                                  c->stream));
    HIP_TRY(c, hipMemcpyAsync(&c->stage->ctl.err, &c->ctl->err, sizeof(int32_t),
                              hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (c->stage->ctl.err & 1) return fail(c, PROT_E_RANGE, "a point coordinate is not finite");
    return PROT_OK;
}

int prot_build_costs(prot_ctx *c, const float *X, const float *Y, int64_t n, int32_t d,
                     double eps, int16_t *k, int64_t ldk, float *m_out)
{
    return prot_build_costs_rect(c, X, n, Y, n, d, eps, k, ldk, m_out);
}

int prot_solve_rounded_rect(prot_ctx *c, const int16_t *k, int64_t n_b, int64_t n_a,
                            int64_t ldk, int64_t T, const prot_opts *o, int32_t warm,
                            int32_t *mate_a, int32_t *mate_b, int32_t *y_a, int32_t *y_b,
                            prot_stats *st)
{
    if (!c) return PROT_E_ARG;
    if (n_b < 0 || n_a < n_b || T < 0 ||
        (n_b > 0 && (!k || ldk < n_a || ldk % 8 || ((uintptr_t)k & 15))) ||
        (n_b > 0 && (!mate_a || !mate_b || !y_a || !y_b)))
        return fail(c, PROT_E_ARG,
                    "prot_solve_rounded: bad pointer, size or alignment (|B| <= |A| required)");
    if (n_a > INT32_MAX / 2) return fail(c, PROT_E_UNSUPPORTED, "n too large");
    if (st) std::memset(st, 0, sizeof(*st));
    if (n_b == 0) return no_rows(c, n_a, warm, mate_a, y_a);
    HIP_TRY(c, hipSetDevice(c->device));
    auto enqueue = [&](bool coop) -> int {
        HIP_TRY(c, prot::launch_clear_err(c->ctl, c->stream));
        HIP_TRY(c, hipEventRecord(c->ev[1], c->stream));
        int r = run_loop(c, k, n_b, n_a, ldk, T, o, warm, mate_a, mate_b, y_a, y_b, kKMaxAccepted,
                         coop);
        if (r) return r;
        HIP_TRY(c, prot::launch_finalize(n_b, mate_b, k, ldk, 0, nullptr, 0, nullptr, nullptr, 0,
                                         c->part_k, c->part_c, c->stream));
        HIP_TRY(c, hipEventRecord(c->ev[4], c->stream));
        return PROT_OK;
    };
    int rc = enqueue(false);
    if (rc || !st) return rc;
    rc = collect(c, st, T, 0.0, 0, false, true);
    if (rc == kRetryCooperative) {
        // a cold start begins again; a warm start's state is as it was given
        if ((rc = enqueue(true))) return rc;
        rc = collect(c, st, T, 0.0, 0, false);
    }
    if (rc) return rc;
    fill_match_counts(c, n_b, st, o);
    return st->status;
}

int prot_solve_rounded(prot_ctx *c, const int16_t *k, int64_t n, int64_t ldk, int64_t T,
                       const prot_opts *o, int32_t warm, int32_t *mate_a, int32_t *mate_b,
                       int32_t *y_a, int32_t *y_b, prot_stats *st)
{
    return prot_solve_rounded_rect(c, k, n, n, ldk, T, o, warm, mate_a, mate_b, y_a, y_b, st);
}

int prot_solve_cost_rect(prot_ctx *c, const float *C, int64_t n_b, int64_t n_a, int64_t ldc,
                         double eps, const prot_opts *o, int32_t *mate_a, int32_t *mate_b,
                         int32_t *y_a, int32_t *y_b, prot_stats *st)
{
    if (!c) return PROT_E_ARG;
    if (n_b < 0 || n_a < n_b ||
        (n_b > 0 && (!C || ldc < n_a || !mate_a || !mate_b || !y_a || !y_b)))
        return fail(c, PROT_E_ARG, "prot_solve_cost: bad pointer or size (|B| <= |A| required)");
    if (!eps_valid(eps_internal(eps, o)))
        return fail(c, PROT_E_EPS, "eps=%g not in (0,1) or too small", eps);
    prot_stats local;
    if (!st) st = &local;
    std::memset(st, 0, sizeof(*st));
    if (n_b == 0) return no_rows(c, n_a, 0, mate_a, y_a);
    HIP_TRY(c, hipSetDevice(c->device));
    const double ei = eps_internal(eps, o);
    const int64_t T = prot_threshold(ei, n_b), ldk = prot_pitch(n_a);
    int k8 = 0;
    int rc = choose_k8(c, o, ei, &k8);
    if (!rc) rc = ensure_matrix(c, n_b, n_a);
    if (rc) return rc;
    HIP_TRY(c, hipEventRecord(c->ev[0], c->stream));
    HIP_TRY(c, prot::launch_round_costs(C, n_b, n_a, ldc, ei, c->kmat, ldk, c->ctl, c->stream,
                                        k8));
    HIP_TRY(c, hipEventRecord(c->ev[1], c->stream));
    const int64_t K = (int64_t)std::floor(1.0 / ei);
    auto enqueue = [&](bool coop) -> int {
        int r = run_loop(c, c->kmat, n_b, n_a, ldk, T, o, 0, mate_a, mate_b, y_a, y_b, K, coop,
                         OnTheFly(), Copies(), k8);
        if (r) return r;
        HIP_TRY(c, prot::launch_finalize(n_b, mate_b, c->kmat, ldk, 1, C, ldc, nullptr, nullptr,
                                         0, c->part_k, c->part_c, c->stream, nullptr, 0.0,
                                         nullptr, k8));
        HIP_TRY(c, hipEventRecord(c->ev[4], c->stream));
        return PROT_OK;
    };
    if ((rc = enqueue(false))) return rc;
    rc = collect(c, st, T, ei, 1, true, true);
    if (rc == kRetryCooperative) {
        if ((rc = enqueue(true))) return rc;
        rc = collect(c, st, T, ei, 1, true);
    }
    if (rc) return rc;
    fill_match_counts(c, n_b, st, o);
    st->kmax = (int32_t)std::floor(1.0 / ei);
    if (c->stage->ctl.err & 1) return fail(c, PROT_E_RANGE, "a cost is NaN or outside [0,1]");
    return st->status;
}

int prot_solve_cost(prot_ctx *c, const float *C, int64_t n, int64_t ldc, double eps,
                    const prot_opts *o, int32_t *mate_a, int32_t *mate_b, int32_t *y_a,
                    int32_t *y_b, prot_stats *st)
{
    return prot_solve_cost_rect(c, C, n, n, ldc, eps, o, mate_a, mate_b, y_a, y_b, st);
}

// The rest of a point-set solve whose loop recomputed its costs and stopped
// to hand over (status 3): the matrix is built, the loop resumes from the
// state in the outputs (a warm start, the same trajectory as one run) and
// the statistics of both parts are added up.
static int hand_over_to_matrix(prot_ctx *c, const float *X, int64_t n_b, const float *Y,
                               int64_t n_a, int32_t d, double ei, int64_t T, int64_t n_max,
                               int64_t ldk, const prot_opts *o, int32_t *mate_a, int32_t *mate_b,
                               int32_t *y_a, int32_t *y_b, prot_stats *st)
{
    const prot_stats first = *st;
    int k8 = 0;
    int rc = choose_k8(c, o, ei, &k8);
    // no room for the matrix: the loop resumes recomputing its costs
    // (PROT_HANDOVER_NO_MATRIX takes that path on purpose, for tests)
    const bool matrix = !std::getenv("PROT_HANDOVER_NO_MATRIX") && !rc && !ensure_matrix(c, n_b, n_a);
    if (!matrix) {
        k8 = 0;
        (void)hipGetLastError();  // (a failed allocation leaves its error behind)
    }
    HIP_TRY(c, hipEventRecord(c->ev[0], c->stream));
    if (matrix) {
        prot::PointsJob j = points_job(c, X, Y, n_b, d, ei, c->kmat, ldk, n_a);
        j.k8 = k8;
        if ((rc = setup_prune(c, j, n_max))) return rc;
        HIP_TRY(c, prot::launch_points(j, n_max, ldk, c->stream));
    }
    HIP_TRY(c, hipEventRecord(c->ev[1], c->stream));
    OnTheFly otf;
    if (!matrix) {
        otf.d = d;
        otf.X = X;
        otf.Y = Y;
        otf.eps = ei;
    }
    prot_opts o2{};
    if (o) o2 = *o;
    o2.max_phases = 0;
    o2.check_warm = 0;
    // the watchdog bounds both parts together
    const int64_t K = (int64_t)std::floor(1.0 / ei);
    const int64_t pb = phase_bound_for(o, n_b, n_a, K, T);
    o2.phase_bound = pb > 0 ? std::max<int64_t>(1, pb - first.phases) : -1;
    rc = run_loop(c, matrix ? c->kmat : nullptr, n_b, n_a, matrix ? ldk : round_up(n_a, 8), T,
                  &o2, 1, mate_a, mate_b, y_a, y_b, K, false, otf, Copies(), k8, first.phases);
    if (rc) return rc;
    if (matrix)
        HIP_TRY(c, prot::launch_finalize(n_b, mate_b, c->kmat, ldk, points_cost_kind(c), nullptr,
                                         0, X, Y, d, c->part_k, c->part_c, c->stream, nullptr, 0.0,
                                         nullptr, k8));
    else
        HIP_TRY(c, prot::launch_finalize(n_b, mate_b, nullptr, 0, 2, nullptr, 0, X, Y, d,
                                         c->part_k, c->part_c, c->stream, &c->ctl->m, ei, c->th));
    HIP_TRY(c, hipEventRecord(c->ev[4], c->stream));
    rc = collect(c, st, T, ei, matrix ? points_cost_kind(c) : 2, true);
    // the phase count the trace reports covers both parts
    const int64_t phases = first.phases + st->phases;
    HIP_TRY(c, hipMemcpyAsync(&c->ctl->phases, &phases, sizeof(int64_t), hipMemcpyHostToDevice,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    st->phases = phases;
    st->sum_free += first.sum_free;
    st->rounds += first.rounds;
    st->max_rounds = std::max(st->max_rounds, first.max_rounds);
    st->scanned += first.scanned;
    st->ms_build += first.ms_build;
    st->ms_loop_kernel += first.ms_loop_kernel;
    st->ms_total += first.ms_total;
    return rc;
}

int prot_solve_points_rect(prot_ctx *c, const float *X, int64_t n_b, const float *Y,
                           int64_t n_a, int32_t d, double eps, const prot_opts *o,
                           int32_t *mate_a, int32_t *mate_b, int32_t *y_a, int32_t *y_b,
                           prot_stats *st)
{
    if (!c) return PROT_E_ARG;
    if (n_b < 0 || n_a < n_b || d < 1 ||
        (n_b > 0 && (!X || !Y || !mate_a || !mate_b || !y_a || !y_b)))
        return fail(c, PROT_E_ARG, "prot_solve_points: bad pointer or size (|B| <= |A| required)");
    if (!eps_valid(eps_internal(eps, o)))
        return fail(c, PROT_E_EPS, "eps=%g not in (0,1) or too small", eps);
    // stats = NULL: enqueue only (no synchronisation, no cooperative retry);
    // prot_ctx_status reports how the solve ended
    const bool enqueue_only = st == nullptr;
    prot_stats local;
    if (!st) st = &local;
    std::memset(st, 0, sizeof(*st));
    if (n_b == 0) return no_rows(c, n_a, 0, mate_a, y_a);
    HIP_TRY(c, hipSetDevice(c->device));
    const double ei = eps_internal(eps, o);
    const int64_t T = prot_threshold(ei, n_b), ldk = prot_pitch(n_a);
    const int64_t n_max = std::max(n_b, n_a);
    const int32_t storage = o ? o->cost_storage : PROT_COSTS_AUTO;
    if (storage < PROT_COSTS_AUTO || storage > PROT_COSTS_ON_THE_FLY)
        return fail(c, PROT_E_ARG, "unknown cost_storage %d", (int)storage);
    if (storage == PROT_COSTS_ON_THE_FLY && d != 2 && d != 3)
        return fail(c, PROT_E_UNSUPPORTED, "costs on the fly need d = 2 or 3 (d = %d)", (int)d);
    if (storage == PROT_COSTS_ON_THE_FLY && c->cost_metric != PROT_METRIC_SQEUCLIDEAN)
        return fail(c, PROT_E_UNSUPPORTED, "costs on the fly take the squared Euclidean cost");
    const bool on_the_fly = storage == PROT_COSTS_ON_THE_FLY ||
                            (storage == PROT_COSTS_AUTO && c->cost_metric == PROT_METRIC_SQEUCLIDEAN &&
                             auto_on_the_fly(d, n_b, n_a));
    int k8 = 0;
    int rc = on_the_fly ? PROT_OK : choose_k8(c, o, ei, &k8);
    if (!rc && !on_the_fly) rc = ensure_matrix(c, n_b, n_a);
    if (!rc) rc = ensure_thresholds(c, ei);
    if (rc) return rc;
    int16_t *kmat = on_the_fly ? nullptr : c->kmat;
    // A loop that recomputes its costs because the matrix would exceed the
    // Infinity Cache hands over to the stored matrix once it has run about
    // twice as many rounds (~10 us each at least) as writing the matrix
    // costs: a long solve pays for the build, a short one never sees it.
    // Only for solves that read their statistics (the host takes the
    // hand-over) and matrices up to 16 GiB (beyond that the recomputation is
    // there for capacity); PROT_AUTO_SWITCH_ROUNDS sets the round (tests).
    uint32_t switch_round = 0;
    const double mat_bytes = 2.0 * (double)n_b * (double)prot_pitch(n_a);
    if (on_the_fly && !enqueue_only && (!o || o->max_phases == 0)) {
        if (const char *e = std::getenv("PROT_AUTO_SWITCH_ROUNDS")) {
            switch_round = (uint32_t)std::max(0, std::atoi(e));
        } else if (storage == PROT_COSTS_AUTO && mat_bytes <= (double)(16ll << 30)) {
            const double build_us = mat_bytes / 3.5e6;
            switch_round = (uint32_t)std::max(16.0, 2.0 * build_us / 10.0);
        }
    }
    // the build's and the whole solve's timing events only when statistics
    // are asked for (each event record holds the next launch back a few us)
    if (!enqueue_only) HIP_TRY(c, hipEventRecord(c->ev[0], c->stream));
    prot::PointsJob j = points_job(c, X, Y, n_b, d, ei, kmat, ldk, n_a);
    j.no_matrix = on_the_fly ? 1 : 0;
    j.k8 = k8;
    if (!on_the_fly && (rc = setup_mfma(c, j, n_max, &c->mfma_buf, &c->mfma_cap))) return rc;
    if ((rc = setup_prune(c, j, n_max))) return rc;
    if ((rc = setup_l1(c, j, n_b, n_a))) return rc;
    HIP_TRY(c, prot::launch_points(j, n_max, ldk, c->stream));
    if (!enqueue_only) HIP_TRY(c, hipEventRecord(c->ev[1], c->stream));
    OnTheFly otf;
    if (on_the_fly) {
        otf.d = d;
        otf.X = X;
        otf.Y = Y;
        otf.eps = ei;
        otf.switch_round = switch_round;
    }
    const int64_t K = (int64_t)std::floor(1.0 / ei);
    auto enqueue = [&](bool coop) -> int {
        int r = run_loop(c, kmat, n_b, n_a, on_the_fly ? round_up(n_a, 8) : ldk, T, o, 0, mate_a,
                         mate_b, y_a, y_b, K, coop, otf, Copies(), k8);
        if (r) return r;
        if (on_the_fly)
            HIP_TRY(c, prot::launch_finalize(n_b, mate_b, nullptr, 0, 2, nullptr, 0, X, Y, d,
                                             c->part_k, c->part_c, c->stream, &c->ctl->m, ei,
                                             c->th));
        else
            HIP_TRY(c, prot::launch_finalize(n_b, mate_b, c->kmat, ldk, points_cost_kind(c),
                                             nullptr, 0, X, Y, d, c->part_k, c->part_c,
                                             c->stream, nullptr, 0.0, nullptr, k8));
        if (!enqueue_only) HIP_TRY(c, hipEventRecord(c->ev[4], c->stream));
        return PROT_OK;
    };
    if ((rc = enqueue(false))) return rc;
    if (enqueue_only) return PROT_OK;
    const int kind = on_the_fly ? 2 : points_cost_kind(c);
    rc = collect(c, st, T, ei, kind, true, true);
    if (rc == kRetryCooperative) {
        if ((rc = enqueue(true))) return rc;
        rc = collect(c, st, T, ei, kind, true);
    }
    if (rc == PROT_OK && st->status == PROT_PARTIAL && c->stage->ctl.status == 3 &&
        !(c->stage->ctl.err & 1))
        rc = hand_over_to_matrix(c, X, n_b, Y, n_a, d, ei, T, n_max, ldk, o, mate_a, mate_b, y_a,
                                 y_b, st);
    if (rc) return rc;
    fill_match_counts(c, n_b, st, o);
    if (c->stage->ctl.err & 1) return fail(c, PROT_E_RANGE, "a point coordinate is not finite");
    return st->status;
}

int prot_solve_points(prot_ctx *c, const float *X, const float *Y, int64_t n, int32_t d,
                      double eps, const prot_opts *o, int32_t *mate_a, int32_t *mate_b,
                      int32_t *y_a, int32_t *y_b, prot_stats *st)
{
    return prot_solve_points_rect(c, X, n, Y, n, d, eps, o, mate_a, mate_b, y_a, y_b, st);
}


namespace {

int ensure_ot(prot_ctx *c, int64_t n_b, int64_t n_a, int64_t cb, int64_t ca)
{
    prot_ctx::Ot &w = c->ot;
    int rc = PROT_OK;
    if (!w.info && (rc = dev_alloc(c, &w.info, 1))) return rc;
    if (n_b > w.cap_b) {
        if ((rc = dev_alloc(c, &w.s_off, (size_t)n_b + 1)) ||
            (rc = dev_alloc(c, &w.ymax, (size_t)n_b)) || (rc = dev_alloc(c, &w.rv, (size_t)n_b)) ||
            (rc = dev_alloc(c, &w.R, (size_t)n_b + 1)))
            return rc;
        w.cap_b = n_b;
    }
    if (n_a > w.cap_a) {
        if ((rc = dev_alloc(c, &w.d_off, (size_t)n_a + 1)) ||
            (rc = dev_alloc(c, &w.qv, (size_t)n_a)) || (rc = dev_alloc(c, &w.Q, (size_t)n_a + 1)))
            return rc;
        w.cap_a = n_a;
    }
    if (n_b * n_a > w.cap_cells) {
        if ((rc = dev_alloc(c, &w.cnt, (size_t)(n_b * n_a)))) return rc;
        w.cap_cells = n_b * n_a;
    }
    if (cb > w.cap_cb) {
        if ((rc = dev_alloc(c, &w.row_pt, (size_t)cb)) || (rc = dev_alloc(c, &w.mate_b, (size_t)cb)) ||
            (rc = dev_alloc(c, &w.y_b, (size_t)cb)))
            return rc;
        w.cap_cb = cb;
    }
    if (ca > w.cap_ca) {
        if ((rc = dev_alloc(c, &w.col_pt, (size_t)ca)) || (rc = dev_alloc(c, &w.mate_a, (size_t)ca)) ||
            (rc = dev_alloc(c, &w.y_a, (size_t)ca)))
            return rc;
        w.cap_ca = ca;
    }
    return PROT_OK;
}

}  // namespace

int prot_ot_solve(prot_ctx *c, const float *C, int64_t n_b, int64_t n_a, int64_t ldc,
                  const double *nu, const double *mu, double eps, const prot_opts *o,
                  double *plan, int64_t ldp, int32_t *y_b_lo, int32_t *y_b_nlo, int32_t *y_a_lo,
                  int32_t *y_a_nlo, prot_ot_stats *st)
{
    if (!c) return PROT_E_ARG;
    if (n_b < 1 || n_a < 1 || !C || ldc < n_a || !nu || !mu || !plan || ldp < n_a || !y_b_lo ||
        !y_b_nlo || !y_a_lo || !y_a_nlo)
        return fail(c, PROT_E_ARG, "prot_ot_solve: bad pointer or size");
    if (n_b > INT32_MAX / 4 || n_a > INT32_MAX / 4)
        return fail(c, PROT_E_UNSUPPORTED, "too many points");
    const double ei = eps_internal(eps, o);
    if (!eps_valid(ei)) return fail(c, PROT_E_EPS, "eps=%g not in (0,1) or too small", eps);
    prot_ot_stats local;
    if (!st) st = &local;
    std::memset(st, 0, sizeof(*st));
    HIP_TRY(c, hipSetDevice(c->device));
    // Section 4: theta = 4n / eps, supplies down, demands up, unit copies
    const double theta = 4.0 * (double)std::max(n_b, n_a) / ei;
    int rc = ensure_ot(c, n_b, n_a, 0, 0);
    if (rc) return rc;
    prot_ctx::Ot &w = c->ot;
    HIP_TRY(c, hipEventRecord(c->ev[0], c->stream));
    HIP_TRY(c, prot::launch_ot_scale(nu, n_b, mu, n_a, theta, w.s_off, w.d_off, w.info,
                                     c->stream));
    HIP_TRY(c, hipMemcpyAsync(&c->stage->ot, w.info, sizeof(prot::OtInfo),
                              hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const prot::OtInfo info = c->stage->ot;
    if (info.err & 1)
        return fail(c, PROT_E_RANGE, "nu and mu must be probability vectors (entries in [0,1], "
                                     "sums within 1e-9 of 1)");
    if (info.err & 2) return fail(c, PROT_E_UNSUPPORTED, "too many copies");
    const int64_t NB = info.copies_b, NA = info.copies_a;
    st->theta = theta;
    st->copies_b = NB;
    st->copies_a = NA;
    int grid = 0;
    bool tg = false;
    if ((rc = grid_for(c, NB, NA, &grid, &tg))) return rc;
    // the copies' columns beyond LDS: prot_ot_solve_clustered is the way
    // (the global column duals serve this path only when forced, as a test)
    if (tg && !c->t_global)
        return fail(c, PROT_E_UNSUPPORTED,
                    "%lld demand copies: their column duals exceed LDS; the clustered "
                    "transport (prot_ot_solve_clustered) has no such limit",
                    (long long)NA);
    if ((rc = ensure_ot(c, n_b, n_a, NB, NA))) return rc;
    if ((rc = ensure_matrix(c, n_b, NA))) return rc;
    const int64_t ldk = prot_pitch(NA);
    HIP_TRY(c, prot::launch_clear_err(c->ctl, c->stream));
    HIP_TRY(c, prot::launch_ot_prepare(C, n_b, n_a, ldc, ei, w.s_off, NB, w.d_off, NA, w.row_pt,
                                       w.col_pt, c->kmat, ldk, w.ymax, c->ctl, c->stream));
    HIP_TRY(c, hipEventRecord(c->ev[1], c->stream));
    const int64_t T = prot_threshold(ei, NB);
    prot_opts lo{};
    if (o) lo = *o;
    lo.no_completion = 0;
    Copies cp;
    cp.rmap = w.row_pt;
    cp.ymax = w.ymax;
    const int64_t K = (int64_t)std::floor(1.0 / ei);
    auto enqueue = [&](bool coop) -> int {
        int r = run_loop(c, c->kmat, NB, NA, ldk, T, &lo, 0, w.mate_a, w.mate_b, w.y_a, w.y_b, K,
                         coop, OnTheFly(), cp);
        if (r) return r;
        prot::OtPlanArgs pa{};
        pa.mate_b = w.mate_b;
        pa.row_pt = w.row_pt;
        pa.col_pt = w.col_pt;
        pa.NB = NB;
        pa.k = c->kmat;
        pa.ldk = ldk;
        pa.cnt = w.cnt;
        pa.n_b = n_b;
        pa.n_a = n_a;
        pa.theta = theta;
        pa.nu = nu;
        pa.mu = mu;
        pa.C = C;
        pa.ldc = ldc;
        pa.plan = plan;
        pa.ldp = ldp;
        pa.rv = w.rv;
        pa.qv = w.qv;
        pa.R = w.R;
        pa.Q = w.Q;
        pa.part_k = c->part_k;
        pa.part_c = c->part_c;
        pa.info = w.info;
        HIP_TRY(c, prot::launch_ot_plan(pa, c->stream));
        HIP_TRY(c, prot::launch_ot_duals(w.y_b, w.s_off, n_b, y_b_lo, y_b_nlo, c->ctl, c->stream));
        HIP_TRY(c, prot::launch_ot_duals(w.y_a, w.d_off, n_a, y_a_lo, y_a_nlo, c->ctl, c->stream));
        HIP_TRY(c, hipEventRecord(c->ev[4], c->stream));
        HIP_TRY(c, hipMemcpyAsync(&c->stage->ot, w.info, sizeof(prot::OtInfo),
                                  hipMemcpyDeviceToHost, c->stream));
        return PROT_OK;
    };
    if ((rc = enqueue(false))) return rc;
    rc = collect(c, &st->loop, T, ei, 1, true, true);  // synchronises the stream
    if (rc == kRetryCooperative) {
        if ((rc = enqueue(true))) return rc;
        rc = collect(c, &st->loop, T, ei, 1, true);
    }
    if (rc) return rc;
    fill_match_counts(c, NB, &st->loop, &lo);
    st->repaired_mass = c->stage->ot.repaired;
    if (c->stage->ctl.err & 1) return fail(c, PROT_E_RANGE, "a cost is NaN or outside [0,1]");
    if (c->stage->ctl.err & 128)
        return fail(c, PROT_E_HIP, "internal: the copies of a point hold more than two duals");
    return st->loop.status;
}

namespace {

int ensure_clusters(prot_ctx *c, int64_t n_b, int64_t n_a)
{
    prot_ctx::Ot &w = c->ot;
    int rc = PROT_OK;
    if (n_b > w.ccap_b) {
        if ((rc = dev_alloc(c, &w.cY, (size_t)n_b)) || (rc = dev_alloc(c, &w.cF, (size_t)n_b)) ||
            (rc = dev_alloc(c, &w.cPF, (size_t)n_b + 1)) ||
            (rc = dev_alloc(c, &w.cact, (size_t)n_b)) || (rc = dev_alloc(c, &w.cneed, (size_t)n_b)) ||
            (rc = dev_alloc(c, &w.cloff, (size_t)n_b)) || (rc = dev_alloc(c, &w.cllen, (size_t)n_b)))
            return rc;
        w.ccap_b = n_b;
    }
    if (n_a > w.ccap_a) {
        if ((rc = dev_alloc(c, &w.cZ, (size_t)n_a)) || (rc = dev_alloc(c, &w.ctop, (size_t)n_a)) ||
            (rc = dev_alloc(c, &w.cbot, (size_t)n_a)) || (rc = dev_alloc(c, &w.cG, (size_t)n_a)) ||
            (rc = dev_alloc(c, &w.cmsum, (size_t)n_a)) ||
            (rc = dev_alloc(c, &w.czt, (size_t)((n_a + 7) & ~7ll))) ||
            (rc = dev_alloc(c, &w.cPG, (size_t)n_a + 1)))
            return rc;
        w.ccap_a = n_a;
    }
    if (n_b * n_a > w.ccap_cells) {
        if ((rc = dev_alloc(c, &w.cw, (size_t)(n_b * n_a))) ||
            (rc = dev_alloc(c, &w.cstage, (size_t)(n_b * n_a + 8))))
            return rc;
        w.ccap_cells = n_b * n_a;
    }
    if (!w.csync && (rc = dev_alloc(c, &w.csync, (size_t)prot::kSyncWords))) return rc;
    const int64_t words = n_a * ((n_b + 63) / 64);
    if (words > w.ccap_mask) {
        if ((rc = dev_alloc(c, &w.cmask, (size_t)words))) return rc;
        w.ccap_mask = words;
    }
    return PROT_OK;
}

}  // namespace

int prot_ot_solve_clustered(prot_ctx *c, const float *C, int64_t n_b, int64_t n_a, int64_t ldc,
                            const double *nu, const double *mu, double eps, const prot_opts *o,
                            double *plan, int64_t ldp, int32_t *y_b_lo, int32_t *y_b_nlo,
                            int32_t *y_a_lo, int32_t *y_a_nlo, prot_ot_stats *st)
{
    if (!c) return PROT_E_ARG;
    if (n_b < 1 || n_a < 1 || !C || ldc < n_a || !nu || !mu || !plan || ldp < n_a || !y_b_lo ||
        !y_b_nlo || !y_a_lo || !y_a_nlo)
        return fail(c, PROT_E_ARG, "prot_ot_solve_clustered: bad pointer or size");
    if (n_b > prot::kClusterMaxPoints || n_a > prot::kClusterMaxPoints)
        return fail(c, PROT_E_UNSUPPORTED, "prot_ot_solve_clustered: at most %lld points a side",
                    (long long)prot::kClusterMaxPoints);
    const double ei = eps_internal(eps, o);
    if (!eps_valid(ei)) return fail(c, PROT_E_EPS, "eps=%g not in (0,1) or too small", eps);
    const int64_t lds_fixed = prot::cluster_lds_fixed(n_b, n_a);
    if (lds_fixed > prot::kClusterLdsBytes)
        return fail(c, PROT_E_UNSUPPORTED, "prot_ot_solve_clustered: the points' state exceeds LDS");
    prot_ot_stats local;
    if (!st) st = &local;
    std::memset(st, 0, sizeof(*st));
    HIP_TRY(c, hipSetDevice(c->device));
    const double theta = 4.0 * (double)std::max(n_b, n_a) / ei;
    int rc = ensure_ot(c, n_b, n_a, 0, 0);
    if (!rc) rc = ensure_clusters(c, n_b, n_a);
    if (!rc) rc = ensure_matrix(c, n_b, n_a);
    if (rc) return rc;
    prot_ctx::Ot &w = c->ot;
    HIP_TRY(c, hipEventRecord(c->ev[0], c->stream));
    HIP_TRY(c, prot::launch_ot_scale(nu, n_b, mu, n_a, theta, w.s_off, w.d_off, w.info,
                                     c->stream));
    HIP_TRY(c, hipMemcpyAsync(&c->stage->ot, w.info, sizeof(prot::OtInfo),
                              hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const prot::OtInfo info = c->stage->ot;
    if (info.err & 1)
        return fail(c, PROT_E_RANGE, "nu and mu must be probability vectors (entries in [0,1], "
                                     "sums within 1e-9 of 1)");
    if (info.err & 2) return fail(c, PROT_E_UNSUPPORTED, "too many copies");
    const int64_t NB = info.copies_b, NA = info.copies_a;
    st->theta = theta;
    st->copies_b = NB;
    st->copies_a = NA;
    const int64_t ldk = prot_pitch(n_a);
    HIP_TRY(c, prot::launch_clear_err(c->ctl, c->stream));
    // eq. (1) on the points' costs
    HIP_TRY(c, prot::launch_round_costs(C, n_b, n_a, ldc, ei, c->kmat, ldk, c->ctl, c->stream));
    HIP_TRY(c, hipEventRecord(c->ev[1], c->stream));
    const int64_t T = prot_threshold(ei, NB);
    const int64_t K = (int64_t)std::floor(1.0 / ei);
    prot::ClusterArgs A{};
    A.k = c->kmat;
    A.ldk = ldk;
    A.n_b = (int32_t)n_b;
    A.n_a = (int32_t)n_a;
    A.s_off = w.s_off;
    A.d_off = w.d_off;
    A.T = T;
    A.origin = o ? o->origin_mode : 0;
    A.max_phases = o ? o->max_phases : 0;
    // the potential of the copies grows by more than T in every phase
    A.phase_bound = phase_bound_for(o, NB, NA, K, T);
    A.G = w.cG;
    A.Yo = w.cY;
    A.Fo = w.cF;
    A.Zo = w.cZ;
    A.topo = w.ctop;
    A.boto = w.cbot;
    A.w = w.cw;
    A.mask = w.cmask;
    A.msum = w.cmsum;
    A.nwb = (int32_t)((n_b + 63) / 64);
    A.act = w.cact;
    A.need = w.cneed;
    A.zt = w.czt;
    A.stage = w.cstage;
    A.loff = w.cloff;
    A.llen = w.cllen;
    A.sync = w.csync;
    A.staged = (int32_t *)(w.csync + prot::kSyncStaged);
    A.PF = w.cPF;
    A.PG = w.cPG;
    A.trace = (long long *)c->trace;
    A.ctl = c->ctl;
    A.lds_bytes = prot::kClusterLdsBytes;
    // PROT_CLUSTER_LIST_CAP: admissible-list entries kept in LDS (a test of
    // the global overflow area)
    if (const char *e = std::getenv("PROT_CLUSTER_LIST_CAP")) {
        const long long cap = std::atoll(e);
        if (cap >= 0) A.lds_bytes = std::min<int64_t>(A.lds_bytes, lds_fixed + 2 * cap);
    }
    HIP_TRY(c, prot::launch_cluster_init(A, c->stream));
    hipEvent_t *le = nullptr;
    if ((rc = next_loop_events(c, &le))) return rc;
    HIP_TRY(c, hipEventRecord(le[0], c->stream));
    int grid = 1;
    HIP_TRY(c, prot::cluster_grid(A.n_b, &grid));
    if (const char *e = std::getenv("PROT_CLUSTER_GRID")) {
        const int g = std::atoi(e);
        if (g >= 1 && g < grid) grid = g;
    }
    HIP_TRY(c, prot::launch_cluster_loop(A, grid, c->stream));
    HIP_TRY(c, hipEventRecord(le[1], c->stream));
    HIP_TRY(c, prot::launch_cluster_counts(A, w.cnt, c->part_k, 1, c->stream));
    prot::OtPlanArgs pa{};
    pa.cnt = w.cnt;
    pa.n_b = n_b;
    pa.n_a = n_a;
    pa.theta = theta;
    pa.nu = nu;
    pa.mu = mu;
    pa.C = C;
    pa.ldc = ldc;
    pa.plan = plan;
    pa.ldp = ldp;
    pa.rv = w.rv;
    pa.qv = w.qv;
    pa.R = w.R;
    pa.Q = w.Q;
    pa.part_k = c->part_k;
    pa.part_c = c->part_c;
    pa.info = w.info;
    HIP_TRY(c, prot::launch_ot_plan_finish(pa, c->stream));
    HIP_TRY(c, prot::launch_cluster_duals(A, y_b_lo, y_b_nlo, y_a_lo, y_a_nlo, c->stream));
    HIP_TRY(c, hipEventRecord(c->ev[4], c->stream));
    HIP_TRY(c, hipMemcpyAsync(&c->stage->ot, w.info, sizeof(prot::OtInfo),
                              hipMemcpyDeviceToHost, c->stream));
    rc = collect(c, &st->loop, T, ei, 1, true);  // synchronises the stream
    if (rc) return rc;
    prot_opts lo{};
    if (o) lo = *o;
    lo.no_completion = 0;
    fill_match_counts(c, NB, &st->loop, &lo);
    st->repaired_mass = c->stage->ot.repaired;
    if (c->stage->ctl.err & 1) return fail(c, PROT_E_RANGE, "a cost is NaN or outside [0,1]");
    if (c->stage->ctl.err & 128)
        return fail(c, PROT_E_HIP, "internal: the copies of a point hold more than two duals");
    return st->loop.status;
}

int32_t prot_batch_max_n(void) { return prot::batch_max_n(); }

int prot_batch_create(prot_ctx *c, int32_t batch, const int64_t *n_host, int32_t d, double eps,
                      const prot_opts *o, prot_batch **out)
{
    return prot_batch_create_config(c, batch, n_host, d, eps, o, nullptr, out);
}

int prot_batch_create_config(prot_ctx *c, int32_t batch, const int64_t *n_host, int32_t d,
                             double eps, const prot_opts *o, const prot_batch_config *cfg,
                             prot_batch **out)
{
    if (!c) return PROT_E_ARG;
    if (!out || batch < 0 || (batch > 0 && !n_host) || d < 1)
        return fail(c, PROT_E_ARG, "prot_batch_create: bad arguments");
    if (cfg && (cfg->engine < PROT_BATCH_ENGINE_AUTO || cfg->engine > PROT_BATCH_ENGINE_TEAMS ||
                cfg->team < 0 || cfg->cost_path < -1 || cfg->cost_path > PROT_COST_AUTO))
        return fail(c, PROT_E_ARG, "prot_batch_create: bad configuration");
    *out = nullptr;
    const double ei = eps_internal(eps, o);
    if (!eps_valid(ei)) return fail(c, PROT_E_EPS, "eps=%g not in (0,1) or too small", eps);
    HIP_TRY(c, hipSetDevice(c->device));
    std::vector<int32_t> n_arr(batch), ldk(batch), order(batch);
    std::vector<int64_t> pt_off(batch), k_off(batch);
    int64_t pts = 0, kel = 0;
    int32_t n_max = 0;
    int64_t ldk_max = 0;
    for (int32_t i = 0; i < batch; ++i) {
        if (n_host[i] < 1 || n_host[i] > prot::batch_max_n())
            return fail(c, PROT_E_UNSUPPORTED, "instance %d: n=%lld outside [1, %d]", i,
                        (long long)n_host[i], prot::batch_max_n());
        n_arr[i] = (int32_t)n_host[i];
        ldk[i] = (int32_t)round_up(n_host[i], 64);
        pt_off[i] = pts;
        k_off[i] = kel;
        pts += n_host[i];
        kel += n_host[i] * ldk[i];
        if (n_arr[i] > n_max) n_max = n_arr[i];
        if (ldk[i] > ldk_max) ldk_max = ldk[i];
        order[i] = i;
    }
    // largest instances first, so the queue ends with short ones
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return n_arr[a] > n_arr[b]; });
    prot_batch *bp = new (std::nothrow) prot_batch();
    if (!bp) return PROT_E_NOMEM;
    bp->ctx = c;
    bp->batch = batch;
    bp->d = d;
    bp->n_max = n_max;
    bp->ldk_max = ldk_max;
    bp->eps = ei;
    if (o) bp->opts = *o;
    bp->kcap = (int32_t)std::floor(1.0 / ei) + 2;
    int rc = PROT_OK;
    if (batch > 0) {
        if (!rc) rc = upload(c, &bp->order, order);
        if (!rc) rc = upload(c, &bp->n_arr, n_arr);
        if (!rc) rc = upload(c, &bp->ldk_arr, ldk);
        if (!rc) rc = upload(c, &bp->pt_off, pt_off);
        if (!rc) rc = upload(c, &bp->k_off, k_off);
        if (!rc) rc = dev_alloc(c, &bp->k, (size_t)kel);
        if (!rc) rc = dev_alloc(c, &bp->m, (size_t)batch);
        if (!rc) rc = dev_alloc(c, &bp->th, (size_t)batch * bp->kcap);
        if (!rc) rc = dev_alloc(c, &bp->stats_tmp, (size_t)batch);
        if (!rc) {
            hipError_t e = prot::batch_grid(n_max, batch, &bp->grid);
            if (e != hipSuccess) rc = hip_fail(c, e, "batch occupancy");
        }
    }
    if (!rc) rc = dev_alloc(c, &bp->err, 1);
    if (!rc) rc = dev_alloc(c, &bp->queue, 1);
    if (!rc && batch > 0)
        rc = dev_alloc(c, &bp->loss_part, (size_t)prot::loss_parts(n_max, d) * batch);
    if (!rc && batch > 0) {
        prot::PointsJob j{};
        j.d = d;
        j.batch = batch;
        const int32_t path = c->cost_path;
        if (cfg && cfg->cost_path >= 0) c->cost_path = cfg->cost_path;
        rc = setup_mfma(c, j, n_max, &bp->mfma_buf, &bp->mfma_cap);
        c->cost_path = path;
        bp->mfma = j.mfma;
    }
    if (!rc && batch > 0) rc = setup_teams(c, bp, n_arr, ldk, pt_off, k_off, cfg);
    if (rc) {
        prot_batch_destroy(bp);
        return rc;
    }
    *out = bp;
    return PROT_OK;
}

int prot_batch_destroy(prot_batch *bp)
{
    if (!bp) return PROT_E_ARG;
    if (bp->ctx) (void)hipSetDevice(bp->ctx->device);
    if (bp->exec) (void)hipGraphExecDestroy(bp->exec);
    if (bp->graph) (void)hipGraphDestroy(bp->graph);
    if (bp->cap_stream) (void)hipStreamDestroy(bp->cap_stream);
    (void)hipFree(bp->order);
    (void)hipFree(bp->n_arr);
    (void)hipFree(bp->ldk_arr);
    (void)hipFree(bp->pt_off);
    (void)hipFree(bp->k_off);
    (void)hipFree(bp->k);
    (void)hipFree(bp->m);
    (void)hipFree(bp->th);
    (void)hipFree(bp->err);
    (void)hipFree(bp->queue);
    (void)hipFree(bp->stats_tmp);
    (void)hipFree(bp->mfma_buf);
    (void)hipFree(bp->loops);
    (void)hipFree(bp->t_key);
    (void)hipFree(bp->t_lists);
    (void)hipFree(bp->t_words);
    (void)hipFree(bp->t_t);
    (void)hipFree(bp->t_ctl);
    (void)hipFree(bp->t_scratch);
    (void)hipFree(bp->t_skip);
    (void)hipFree(bp->loss_part);
    delete bp;
    return PROT_OK;
}

int prot_batch_run(prot_batch *bp, const float *X, const float *Y, int32_t *mate_a,
                   int32_t *mate_b, int32_t *y_a, int32_t *y_b, prot_instance_stats *stats)
{
    if (!bp) return PROT_E_ARG;
    prot_ctx *c = bp->ctx;
    if (bp->batch == 0) return PROT_OK;
    if (!batch_args_ok(bp, X, Y, mate_a, mate_b, y_a, y_b))
        return fail(c, PROT_E_ARG, "prot_batch_run: null pointer");
    HIP_TRY(c, hipSetDevice(c->device));
    return batch_enqueue(bp, c->stream, X, Y, mate_a, mate_b, y_a, y_b, stats);
}

int prot_batch_autotune(prot_ctx *c, int32_t batch, const int64_t *n_host, int32_t d,
                        double eps, const prot_opts *o, const float *X, const float *Y,
                        int32_t reps, prot_batch_config *best, double *best_ms, int32_t *tried)
{
    if (!c) return PROT_E_ARG;
    if (batch < 1 || !n_host || !X || !Y || !best || reps < 1)
        return fail(c, PROT_E_ARG, "prot_batch_autotune: bad arguments");
    HIP_TRY(c, hipSetDevice(c->device));
    int64_t total = 0, n_max = 0;
    for (int32_t i = 0; i < batch; ++i) {
        total += n_host[i];
        n_max = std::max<int64_t>(n_max, n_host[i]);
    }
    // the candidates: the LDS engine, teams of every size, each cost path
    std::vector<prot_batch_config> cand;
    const int paths = d >= prot::kMfmaMinD ? 2 : 1;
    for (int path = 0; path < paths; ++path) {
        cand.push_back(prot_batch_config{PROT_BATCH_ENGINE_LDS, 0, path, 0});
        for (int team = 1; team <= 8; ++team)
            if (team * 1024 >= n_max) cand.push_back(prot_batch_config{PROT_BATCH_ENGINE_TEAMS, team, path, 0});
    }
    int32_t *out = nullptr;
    int rc = dev_alloc(c, &out, (size_t)(4 * total));
    if (rc) return rc;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipFree(out);
        if (e0) (void)hipEventDestroy(e0);
        return fail(c, PROT_E_HIP, "event creation failed");
    }
    double best_t = -1.0;
    int32_t count = 0;
    for (const prot_batch_config &cf : cand) {
        prot_batch *bp = nullptr;
        if (prot_batch_create_config(c, batch, n_host, d, eps, o, &cf, &bp) != PROT_OK) continue;
        int r = prot_batch_run(bp, X, Y, out, out + total, out + 2 * total, out + 3 * total,
                               nullptr);
        float ms = 0.0f;
        if (r == PROT_OK && hipEventRecord(e0, c->stream) == hipSuccess) {
            for (int i = 0; i < reps && r == PROT_OK; ++i)
                r = prot_batch_run(bp, X, Y, out, out + total, out + 2 * total, out + 3 * total,
                                   nullptr);
            if (r == PROT_OK && (hipEventRecord(e1, c->stream) != hipSuccess ||
                                 hipEventSynchronize(e1) != hipSuccess ||
                                 hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                r = PROT_E_HIP;
        }
        prot_batch_destroy(bp);
        if (r != PROT_OK) continue;
        count += 1;
        const double t = (double)ms / reps;
        if (best_t < 0.0 || t < best_t) {
            best_t = t;
            *best = cf;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(out);
    if (tried) *tried = count;
    if (best_ms) *best_ms = best_t;
    if (count == 0) return fail(c, PROT_E_UNSUPPORTED, "no configuration ran");
    return PROT_OK;
}

int prot_batch_capture(prot_batch *bp, const float *X, const float *Y, int32_t *mate_a,
                       int32_t *mate_b, int32_t *y_a, int32_t *y_b, prot_instance_stats *stats)
{
    if (!bp) return PROT_E_ARG;
    prot_ctx *c = bp->ctx;
    if (bp->batch == 0) return PROT_OK;
    if (!batch_args_ok(bp, X, Y, mate_a, mate_b, y_a, y_b))
        return fail(c, PROT_E_ARG, "prot_batch_capture: null pointer");
    HIP_TRY(c, hipSetDevice(c->device));
    if (!bp->cap_stream)
        HIP_TRY(c, hipStreamCreateWithFlags(&bp->cap_stream, hipStreamNonBlocking));
    if (bp->exec) {
        (void)hipGraphExecDestroy(bp->exec);
        bp->exec = nullptr;
    }
    if (bp->graph) {
        (void)hipGraphDestroy(bp->graph);
        bp->graph = nullptr;
    }
    HIP_TRY(c, hipStreamBeginCapture(bp->cap_stream, hipStreamCaptureModeThreadLocal));
    const int rc = batch_enqueue(bp, bp->cap_stream, X, Y, mate_a, mate_b, y_a, y_b, stats);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(bp->cap_stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
    bp->graph = g;
    HIP_TRY(c, hipGraphInstantiate(&bp->exec, bp->graph, nullptr, nullptr, 0));
    return PROT_OK;
}

int prot_batch_replay(prot_batch *bp)
{
    if (!bp) return PROT_E_ARG;
    prot_ctx *c = bp->ctx;
    if (bp->batch == 0) return PROT_OK;
    if (!bp->exec) return fail(c, PROT_E_ARG, "prot_batch_replay: nothing captured");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipGraphLaunch(bp->exec, c->stream));
    return PROT_OK;
}

int prot_batch_loss_fwd(prot_batch *bp, const float *X, const float *Y, const int32_t *mate_b,
                        float *loss)
{
    if (!bp) return PROT_E_ARG;
    prot_ctx *c = bp->ctx;
    if (bp->batch == 0) return PROT_OK;
    if (!X || !Y || !mate_b || !loss) return fail(c, PROT_E_ARG, "prot_batch_loss_fwd: null pointer");
    HIP_TRY(c, hipSetDevice(c->device));
    prot::LossArgs a{bp->batch, bp->d, bp->n_arr, bp->pt_off, X, Y, nullptr, mate_b, 0};
    HIP_TRY(c, prot::launch_loss_fwd(a, bp->n_max, bp->loss_part, loss, c->stream));
    return PROT_OK;
}

int prot_batch_loss_bwd(prot_batch *bp, const float *X, const float *Y, const int32_t *mate_a,
                        const int32_t *mate_b, const float *grad_loss, float *dX, float *dY)
{
    if (!bp) return PROT_E_ARG;
    prot_ctx *c = bp->ctx;
    if (bp->batch == 0) return PROT_OK;
    if (!X || !Y || !mate_a || !mate_b || !grad_loss || !dX || !dY)
        return fail(c, PROT_E_ARG, "prot_batch_loss_bwd: null pointer");
    HIP_TRY(c, hipSetDevice(c->device));
    prot::LossArgs a{bp->batch, bp->d, bp->n_arr, bp->pt_off, X, Y, mate_a, mate_b, 0};
    HIP_TRY(c, prot::launch_loss_bwd(a, bp->n_max, grad_loss, dX, dY, c->stream));
    return PROT_OK;
}

int prot_solve_batched_points(prot_ctx *c, int32_t batch, const int64_t *n_host, int32_t d,
                              const float *X, const float *Y, double eps, const prot_opts *o,
                              int32_t *mate_a, int32_t *mate_b, int32_t *y_a, int32_t *y_b,
                              prot_instance_stats *stats_host)
{
    if (!c) return PROT_E_ARG;
    prot_batch *bp = nullptr;
    int rc = prot_batch_create(c, batch, n_host, d, eps, o, &bp);
    if (rc) return rc;
    rc = prot_batch_run(bp, X, Y, mate_a, mate_b, y_a, y_b, nullptr);
    int32_t err = 0;
    if (!rc && batch > 0) {
        hipError_t e = hipMemcpyAsync(&err, bp->err, sizeof(int32_t), hipMemcpyDeviceToHost,
                                      c->stream);
        if (e == hipSuccess && stats_host)
            e = hipMemcpyAsync(stats_host, bp->stats_tmp, sizeof(prot_instance_stats) * batch,
                               hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) rc = hip_fail(c, e, "batched solve");
    }
    prot_batch_destroy(bp);
    if (!rc) rc = batch_err_status(c, err);
    return rc;
}

int prot_ctx_status(prot_ctx *c)
{
    if (!c) return PROT_E_ARG;
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipMemcpyAsync(&c->stage->ctl, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    const Ctl &h = c->stage->ctl;
    if (h.err & 1) return fail(c, PROT_E_RANGE, "a cost or coordinate is NaN or out of range");
    if (h.err & 2) return fail(c, PROT_E_STATE, "invalid warm-start state");
    return loop_status(c, h);
}

int prot_batch_status(prot_batch *bp)
{
    if (!bp) return PROT_E_ARG;
    prot_ctx *c = bp->ctx;
    if (bp->batch == 0) return PROT_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipMemcpyAsync(&c->stage->ctl.err, bp->err, sizeof(int32_t),
                              hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return batch_err_status(c, c->stage->ctl.err);
}

int prot_ot_loss_fwd(prot_ctx *c, int32_t batch, int64_t n, int32_t d, const float *X,
                     const float *Y, const int32_t *mate_b, float *loss)
{
    if (!c) return PROT_E_ARG;
    if (batch < 0 || n < 0 || d < 1 || (batch > 0 && n > 0 && (!X || !Y || !mate_b || !loss)))
        return fail(c, PROT_E_ARG, "prot_ot_loss_fwd: bad pointer or size");
    if (batch == 0) return PROT_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    const int64_t need = (int64_t)prot::loss_parts(n, d) * batch;
    if (need > c->loss_cap || !c->loss_part) {
        const int rc = dev_alloc(c, &c->loss_part, (size_t)need);
        if (rc) return rc;
        c->loss_cap = need;
    }
    prot::LossArgs a{batch, d, nullptr, nullptr, X, Y, nullptr, mate_b, n};
    HIP_TRY(c, prot::launch_loss_fwd(a, n, c->loss_part, loss, c->stream));
    return PROT_OK;
}

int prot_ot_loss_fwd_static(int32_t batch, int64_t n, int32_t d, const float *X, const float *Y,
                            const int32_t *mate_b, float *loss, void *hip_stream)
{
    auto bad = [](int code, const std::string &msg) {
        g_free_err = msg;
        return code;
    };
    if (batch < 0 || n < 0 || d < 1 || (batch > 0 && n > 0 && (!X || !Y || !mate_b || !loss)))
        return bad(PROT_E_ARG, "prot_ot_loss_fwd_static: bad pointer or size");
    if (batch == 0) return PROT_OK;
    const int64_t need = (int64_t)prot::loss_parts(n, d) * batch;
    if (need > prot::kStaticLossParts)
        return bad(PROT_E_UNSUPPORTED,
                   "prot_ot_loss_fwd_static: " + std::to_string(batch) + " instances need " +
                       std::to_string(need) + " partial sums; the fixed array holds " +
                       std::to_string(prot::kStaticLossParts));
    double *partial = nullptr;
    hipError_t e = prot::static_loss_partials(&partial);
    if (e != hipSuccess)
        return bad(PROT_E_HIP, std::string("prot_ot_loss_fwd_static: address of the fixed "
                                           "array: ") + hipGetErrorString(e));
    prot::LossArgs a{batch, d, nullptr, nullptr, X, Y, nullptr, mate_b, n};
    e = prot::launch_loss_fwd(a, n, partial, loss, (hipStream_t)hip_stream);
    if (e != hipSuccess)
        return bad(PROT_E_HIP, std::string("prot_ot_loss_fwd_static: launch: ") +
                                   hipGetErrorString(e));
    return PROT_OK;
}

int prot_ot_loss_bwd(prot_ctx *c, int32_t batch, int64_t n, int32_t d, const float *X,
                     const float *Y, const int32_t *mate_b, const float *grad_loss, float *dX,
                     float *dY)
{
    if (!c) return PROT_E_ARG;
    if (batch < 0 || n < 0 || d < 1 ||
        (batch > 0 && n > 0 && (!X || !Y || !mate_b || !grad_loss || !dX || !dY)))
        return fail(c, PROT_E_ARG, "prot_ot_loss_bwd: bad pointer or size");
    if (batch == 0 || n == 0) return PROT_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    prot::LossArgs a{batch, d, nullptr, nullptr, X, Y, nullptr, mate_b, n};
    HIP_TRY(c, prot::launch_loss_bwd(a, n, grad_loss, dX, dY, c->stream));
    return PROT_OK;
}

int64_t prot_get_round_times(prot_ctx *c, int64_t *out, int64_t cap)
{
    if (!c || !out || cap < 0) return PROT_E_ARG;
    if (!c->rtime) return 0;
    Ctl h;
    if (hipMemcpyAsync(&c->stage->ctl, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream) !=
            hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return PROT_E_HIP;
    h = c->stage->ctl;
    (void)h;
    int64_t m = cap < prot::kRoundTimeCap ? cap : prot::kRoundTimeCap;
    if (hipMemcpyAsync(out, c->rtime, sizeof(int64_t) * 3 * (size_t)m, hipMemcpyDeviceToHost,
                       c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return PROT_E_HIP;
    return m;
}

int32_t prot_loop_times(prot_ctx *c, float *ms_out, int32_t count)
{
    if (!c || count < 0 || (count > 0 && !ms_out)) return PROT_E_ARG;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return PROT_E_HIP;
    int64_t m = std::min<int64_t>({(int64_t)count, c->loop_launches,
                                   (int64_t)prot_ctx::kLoopEvents});
    for (int64_t i = 0; i < m; ++i) {
        // oldest first: the latest launch goes last
        const int slot = (int)((c->loop_slot - (m - 1 - i) + 2 * prot_ctx::kLoopEvents) %
                               prot_ctx::kLoopEvents);
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, c->loop_ev[slot][0], c->loop_ev[slot][1]) != hipSuccess)
            return fail(c, PROT_E_HIP, "prot_loop_times: an event was not recorded");
        ms_out[i] = ms;
    }
    return (int32_t)m;
}

int64_t prot_get_trace(prot_ctx *c, int64_t *out, int64_t cap)
{
    if (!c || !out || cap < 0) return PROT_E_ARG;
    Ctl h;
    if (hipMemcpyAsync(&c->stage->ctl, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream) !=
            hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return PROT_E_HIP;
    h = c->stage->ctl;
    int64_t m = h.phases;
    if (m > prot::kTraceCap) m = prot::kTraceCap;
    if (m > cap) m = cap;
    if (m > 0) {
        if (hipMemcpyAsync(out, c->trace, sizeof(int64_t) * 4 * (size_t)m, hipMemcpyDeviceToHost,
                           c->stream) != hipSuccess ||
            hipStreamSynchronize(c->stream) != hipSuccess)
            return PROT_E_HIP;
    }
    return m;
}

}  // extern "C"
