// Internal declarations shared by the HIP translation units of libprot.
// Not part of the public C ABI (see include/prot.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cost_common.h"

namespace prot {

// Device-side control block of one phase loop. Zeroed by the reset kernel.
struct alignas(128) Ctl {
    uint32_t gate_count;          // phase loop, plain launch: tickets handed out
    uint32_t gate;                // 0 open; else kGateClosed | workgroups taking part
    unsigned long long pad2[2];
    uint32_t free0;               // |B'| of the first phase (set by the init kernel)
    uint32_t tag_last;            // last list tag used by a launch (kept across launches,
                                  // so that no entry of an earlier launch matches a tag)
    unsigned long long pad1[2];
    unsigned long long scanned;   // matrix entries examined
    int32_t status;               // 0 finished, 1 stopped at max_phases, 2 stopped by the
                                  // phase-bound watchdog
    int32_t err;                  // bit 0: cost out of range / non-finite; bit 1: bad state;
                                  // bit 2: a list entry did not arrive; bit 3: round ids exhausted;
                                  // bit 4: too few workgroups resident for the rows (nothing ran);
                                  // bit 5: a round barrier timed out; bit 6: a dual left its
                                  // 15-bit field; bit 7: transport copies hold > 2 duals
    int64_t phases;
    int64_t sum_free;
    int64_t rounds;
    int64_t max_rounds;
    int64_t free_after;           // |free B| when the loop stopped
    int32_t kmax;                 // largest rounded cost produced by a cost build
    int32_t pad;
    float m;                      // max squared distance of the last point build
};

// Error bits of a phase loop that leave its state unusable.
constexpr int32_t kErrLoop = 4 | 8 | 32 | 64;
constexpr int kLoopThreads = 1024;      // threads per workgroup of the loop
// Round barrier: the workgroups are split into up to kMaxGroups groups
// (blockIdx % G); each round has one word per group, kWordStride words
// apart (one 128-byte line each), in a ring of three rounds: round r uses
// words[(r % 3) * kMaxGroups * kWordStride + g * kWordStride]. Workgroup 0
// clears the words of round r + 1 during round r, after every reader of
// their previous use (round r - 2) has passed a barrier. Each list of the
// loop is split into G regions of list_cap entries, one per group.
constexpr int kMaxGroups = 32;
constexpr int kWordStride = 16;
constexpr int kTraceCap = 65536;        // phases recorded in the trace
constexpr int kFinalizeBlocks = 256;    // partial sums of the finalize kernel
// Per-block maxima of the single-instance maximum pass (d = 2, 3): at most
// max(kMaxParts, ceil(columns / 256)) of them; the pruned pass stores
// kPairsMaxBlocks.
constexpr int kMaxParts = 2048;
constexpr int kPairsMaxBlocks = 1024;
inline int64_t max_parts_cap(int64_t n_max)
{
    const int64_t cols = (n_max + 255) / 256;
    return cols > kMaxParts ? cols : kMaxParts;
}
constexpr int kRoundTimeCap = 65536;    // rounds recorded by the round timer

struct LoopArgs {
    const int16_t *k;
    int64_t ldk;
    int32_t n;              // rows |B|
    int32_t n_pad;          // n_a rounded up to 8 (LDS dual array length)
    int32_t n_a;            // columns |A| >= |B| (Section 3.3; = n when balanced)
    int32_t wide;           // 1: rows travel in 18 bits (n > 131,071; duals <= 16,383)
    int64_t T;
    int32_t origin;         // 0: diagonal, 1: zero
    // stop with status 3 at the first phase start from this round on (0:
    // never): a loop that recomputes its costs hands over to the stored
    // matrix once it has run long enough to pay for building it
    uint32_t switch_round;
    int64_t max_phases;
    int64_t phase_bound;      // watchdog: stop with status 2 after this many phases (0: none)
    int64_t barrier_ticks;    // bounded round-barrier wait, 100 MHz ticks (0: the default)
    unsigned long long *key;  // per column: round, row and row dual of its last winner
    uint16_t *t;              // per column: -y(a) (number of phases it was taken in)
    int32_t *y_b;
    unsigned long long *F[2]; // free lists B', (phase tag << 32) | row (ping-pong by parity)
    unsigned long long *L[2]; // columns taken in a phase, (phase tag << 32) | column
    int64_t list_cap;         // entries per group region of F and L (>= n)
    int32_t groups;           // G, 1 <= G <= min(kMaxGroups, grid)
    int32_t pad2;
    unsigned long long *words;  // round words, 3 * kMaxGroups * kWordStride
    int64_t y_off;            // batched teams: y_b is the launch's y_b base + y_off
    Ctl *ctl;
    int64_t *trace;           // 4 int64 per phase
    int64_t *rtime;           // optional: 3 int64 per round (see kRoundTimeCap)
    // Matrix-free (pd = 2 or 3): k is computed from the points instead of read
    // from k; m, the threshold table and eps are those of the cost build.
    // Exact fast-forward (null: off): skip[b] > 0 means row b cannot find an
    // admissible column in its next skip[b] phases (its smallest slack, seen
    // by a full first-round scan that found none, was skip[b] + 1 or more).
    uint32_t *skip;
    int32_t pd;               // 0: read k
    int32_t k8;               // 1: k is a uint8 matrix (K <= 253; padding 0xFF)
    const float *px, *py;     // n x pd rows (supply) and columns (demand)
    const float *pm;          // device: max squared distance
    const float *pth;         // device: threshold table th[0..K+1]
    double peps;
    // Copies of the transport reduction (null: off). Row b reads the cost row
    // rmap[b] (the supply point it copies). A free row's dual is raised to the
    // largest dual of its point's copies when the row enters a phase and when
    // the loop ends; ymax[p] = ((q + 1) << 32) | m holds that largest dual m
    // as it was after phase q, the last phase in which one of p's copies
    // found no column (initially (0 << 32) | 1). Every copy in B' was raised,
    // so all that phase's copies of p end at the same m; a reader in phase q
    // itself takes m - 1.
    const int32_t *rmap;
    unsigned long long *ymax;
    // 1: a plain launch whose resident workgroups agree on how many take part
    // (Ctl::gate); 0: a cooperative launch. gate_cap > 0 closes the gate at
    // that many workgroups (a test of the partial case).
    int32_t gated, gate_cap;
    // Column duals in global memory (null: in LDS): each workgroup keeps its
    // copy of t in tpriv + blockIdx.x * n_pad, for columns beyond LDS.
    uint16_t *tpriv;
};
constexpr uint32_t kGateClosed = 0x80000000u;

// Per-instance results of the batched solver (layout of prot_instance_stats).
struct InstanceStats {
    int64_t phases, sum_free, rounds, max_rounds, scanned, matched_in_phases,
        completed_pairs, sum_k, threshold;
    int32_t status, kmax;
    double cost, cost_scale;
};

struct BatchArgs {
    int32_t batch;
    int32_t d;
    double eps;
    int64_t max_phases;
    int32_t origin;
    int32_t complete;
    const int32_t *order;     // instance ids, largest n first
    const int32_t *n_arr;
    const int32_t *ldk_arr;
    const int64_t *pt_off;    // first row of each instance in X, Y and the outputs
    const int64_t *k_off;     // element offset of each instance's rounded costs
    const int16_t *k;
    const float *X, *Y, *m;
    int32_t *mate_a, *mate_b, *y_a, *y_b;
    InstanceStats *stats;
    unsigned int *queue;
    int64_t *rtime;           // optional diagnostics: 4 int64 per round of the first job
    int32_t *err;             // bit 8: an instance was stopped by the phase-bound watchdog
};

// Batched instances solved by teams of phase-loop workgroups: per-instance
// loop arguments on the device, plus what the set-up and the finish need.
struct TeamArgs {
    int32_t batch;
    int32_t d;
    int32_t complete;
    int32_t pad;
    double eps;
    const LoopArgs *loops;    // per instance
    const int64_t *pt_off;    // first row of each instance in X, Y and the outputs
    const float *X, *Y, *m;
    int32_t *mate_a, *mate_b, *y_a, *y_b;
    int32_t *scratch;         // 2 * (sum of n) ints; instance i at 2 * pt_off[i]
    InstanceStats *stats;
    int32_t *err;             // bits 2 and 3 of a loop's error word are collected here
};

struct LossArgs {
    int32_t batch;
    int32_t d;
    const int32_t *n_arr;     // per-instance n (null: every instance has n_uniform)
    const int64_t *pt_off;    // first row of each instance (null: inst * n_uniform)
    const float *X, *Y;
    const int32_t *mate_a, *mate_b;  // mate_a null: the backward scatters through mate_b
    int64_t n_uniform;
};

// cost.hip
hipError_t launch_round_costs(const float *C, int64_t n, int64_t na, int64_t ldc, double eps,
                              int16_t *k, int64_t ldk, Ctl *ctl, hipStream_t s, int k8 = 0);
hipError_t launch_points(const PointsJob &j, int64_t n_max, int64_t ldk_max, hipStream_t s);

// cost_mfma.hip
constexpr int32_t kMfmaMinD = 16;          // d from which the matrix cores can be used
constexpr int32_t kMfmaAutoD = 48;         // d from which PROT_COST_AUTO uses them
constexpr int64_t kMfmaTile = 128;      // tile rows and columns of the matrix-core build
float mfma_error_constant(int32_t d);
hipError_t launch_points_mfma(const PointsJob &j, const MfmaAux &x, int64_t n_max,
                              int64_t ldk_max, hipStream_t s);

// batch.hip
int32_t batch_max_n();
hipError_t batch_grid(int32_t n_max, int32_t batch, int *grid);
hipError_t launch_batch_solve(const BatchArgs &a, int32_t n_max, int grid, hipStream_t s);

// loss.hip
// partial: loss_parts(n_max, d) * batch doubles of workspace.
int loss_parts(int64_t n_max, int32_t d);
hipError_t launch_loss_fwd(const LossArgs &a, int64_t n_max, double *partial, float *loss,
                           hipStream_t s);
// Partial sums (instances x blocks) that prot_ot_loss_fwd_static can hold in
// the library's fixed array (512 KiB per device).
constexpr int64_t kStaticLossParts = 65536;
hipError_t static_loss_partials(double **out);
hipError_t launch_loss_bwd(const LossArgs &a, int64_t n_max, const float *grad_loss, float *dX,
                           float *dY, hipStream_t s);

// solve.hip
hipError_t launch_init(const LoopArgs &a, int32_t warm, const int32_t *mate_a,
                       int32_t *mate_b, const int32_t *y_a, hipStream_t s);
hipError_t launch_clear_err(Ctl *ctl, hipStream_t s, int32_t mask = -1);
hipError_t launch_check_state(int64_t n, int64_t na, const int32_t *mate_a,
                              const int32_t *mate_b, const int32_t *y_a, const int32_t *y_b,
                              int32_t ybound, Ctl *ctl, hipStream_t s);
hipError_t launch_check_feasible(const int16_t *k, int64_t ldk, int64_t n, int64_t na,
                                 const int32_t *mate_b, const int32_t *y_a, const int32_t *y_b,
                                 Ctl *ctl, hipStream_t s);
hipError_t loop_grid(int32_t n_pad, int wgs_per_cu, int *grid_max);
hipError_t loop_grid_tg(int wgs_per_cu, int *grid_max);  // column duals in global memory
hipError_t launch_clear_times(int64_t *rtime, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t s);
// ev_start / ev_stop (may be null) take the loop launch's start and end.
hipError_t launch_loop(const LoopArgs &a, int grid, hipStream_t s, hipEvent_t ev_start,
                       hipEvent_t ev_stop);
// Teams: workgroups a cooperative launch of the multi-instance loop can hold.
hipError_t loop_grid_multi(int32_t n_pad_max, int wgs_per_cu, int *grid_max);
hipError_t launch_team_init(const TeamArgs &t, int32_t n_pad_max, hipStream_t s);
hipError_t launch_loop_multi(const LoopArgs *arr, int count, int team, int32_t n_pad_max,
                             int32_t *y_base, hipStream_t s);
hipError_t launch_team_finish(const TeamArgs &t, hipStream_t s);
hipError_t launch_finish(const LoopArgs &a, int32_t warm, int32_t complete,
                         int32_t *mate_a, int32_t *mate_b, int32_t *y_a, int32_t *scratch,
                         hipStream_t s);
// cost_kind: 0 none, 1 cost matrix C (ldc), 2 points X, Y (d) with scale m.
// With k == nullptr (points, costs on the fly) the rounded cost of each
// matched pair is recomputed from the points, *m_dev, eps and th.
hipError_t launch_finalize(int64_t n, const int32_t *mate_b, const int16_t *k,
                           int64_t ldk, int cost_kind, const float *C, int64_t ldc,
                           const float *X, const float *Y, int32_t d,
                           long long *part_k, double *part_c, hipStream_t s,
                           const float *m_dev = nullptr, double eps = 0.0,
                           const float *th = nullptr, int k8 = 0);

// Optimal transport through copies (Section 4).
struct OtInfo {
    long long copies_b, copies_a;  // sum floor(theta nu_b), sum ceil(theta mu_a)
    int32_t err;                   // 1: masses not probability vectors; 2: too many copies
    int32_t pad;
    double repaired;               // mass moved by the feasibility repair
};

struct OtPlanArgs {
    const int32_t *mate_b;         // copy level, NB entries
    const int32_t *row_pt, *col_pt;
    int64_t NB;
    const int16_t *k;              // expanded rounded costs, n_b x ldk
    int64_t ldk;
    int32_t *cnt;                  // n_b x n_a pair counts
    int64_t n_b, n_a;
    double theta;
    const double *nu, *mu;
    const float *C;
    int64_t ldc;
    double *plan;
    int64_t ldp;
    double *rv, *qv;               // left to send (n_b), room left (n_a)
    double *R, *Q;                 // their running totals (n_b + 1, n_a + 1)
    long long *part_k;
    double *part_c;
    OtInfo *info;
};

hipError_t launch_ot_scale(const double *nu, int64_t n_b, const double *mu, int64_t n_a,
                           double theta, int64_t *s_off, int64_t *d_off, OtInfo *info,
                           hipStream_t s);
hipError_t launch_ot_prepare(const float *C, int64_t n_b, int64_t n_a, int64_t ldc, double eps,
                             const int64_t *s_off, int64_t NB, const int64_t *d_off, int64_t NA,
                             int32_t *row_pt, int32_t *col_pt, int16_t *k, int64_t ldk,
                             unsigned long long *ymax, Ctl *ctl, hipStream_t s);
hipError_t launch_ot_plan(const OtPlanArgs &a, hipStream_t s);
// The plan from pair counts already in a.cnt (column, row, running totals, route).
hipError_t launch_ot_plan_finish(const OtPlanArgs &a, hipStream_t s);
hipError_t launch_ot_duals(const int32_t *y, const int64_t *off, int64_t n_pts, int32_t *lo,
                           int32_t *nlo, Ctl *ctl, hipStream_t s);

// ot_cluster.hip: transport with the copies kept as clusters (Lemma 4.1).
constexpr int64_t kClusterMaxPoints = 4096;   // points per side (one workgroup)
constexpr int64_t kClusterLdsBytes = 159 * 1024;
constexpr int kSyncWords = 256;              // hand-over words of the cluster loop
constexpr int kSyncStaged = 128;             // the word counting staged list entries
struct ClusterArgs {
    const int16_t *k;              // n_b x ldk rounded costs of the points
    int64_t ldk;
    int32_t n_b, n_a;
    const int64_t *s_off, *d_off;  // copy offsets (n + 1 entries each)
    int64_t T;                     // stop once at most T supply copies are free
    int32_t origin;                // 0: scan of b from column b mod n_a; 1: from 0
    int64_t max_phases;            // 0: no limit (status 1 when reached)
    int64_t phase_bound;           // watchdog (status 2 when reached; 0: none)
    int32_t *G;                    // n_a: free demand copies
    int32_t *Yo, *Fo;              // n_b: final Y and free copies
    int32_t *Zo, *topo, *boto;     // n_a: final Z and copies at Z and Z - 1
    int2 *w;                       // n_b x n_a pair counts by parity of the demand level
    unsigned long long *mask;      // n_a x nwb: supply points with a pair
    unsigned long long *msum;      // n_a: bit i set iff word i of the point's mask is nonzero
    int32_t nwb;
    // the phase's lists, built by every workgroup of the loop
    int32_t *act, *need;           // n_b: rows with free copies, their Y - 1
    int32_t *zt;                   // n_a rounded up to 8: top level, or a never-met level
    uint16_t *stage;               // n_b x n_a + 8: the lists, one block per row
    int32_t *loff, *llen;          // n_b: a row's block
    uint32_t *sync;                // kSyncWords hand-over words
    int32_t *staged;               // = sync + kSyncStaged: entries staged
    int64_t *PF, *PG;              // running totals of F and G (n_b + 1, n_a + 1)
    long long *trace;              // kTraceCap x 4 per-phase record, or null
    Ctl *ctl;
    int64_t lds_bytes;             // dynamic LDS of the loop
};
int64_t cluster_lds_fixed(int64_t n_b, int64_t n_a);
hipError_t launch_cluster_init(const ClusterArgs &A, hipStream_t s);
hipError_t cluster_grid(int32_t n_b, int *grid);  // workgroups of the loop
hipError_t launch_cluster_loop(const ClusterArgs &A, int grid, hipStream_t s);
hipError_t launch_cluster_counts(const ClusterArgs &A, int32_t *cnt, long long *part_k,
                                 int complete, hipStream_t s);
hipError_t launch_cluster_duals(const ClusterArgs &A, int32_t *b_lo, int32_t *b_nlo,
                                int32_t *a_lo, int32_t *a_nlo, hipStream_t s);

}  // namespace prot
