// Many independent assignment instances in one launch (the same phase loop
// as solve.hip, arXiv:2203.03732 Section 2.2, with the same proposal rounds
// and tie-break, so every instance's result is identical to a
// single-instance solve on its rounded costs).
//
// Each workgroup pops instances from a queue (largest n first) and solves an
// instance alone: the column keys, the duals, the free and taken lists and
// the active rows of a round all live in LDS, the round barrier is
// __syncthreads, and only the rounded-cost matrix (built beforehand by the
// batched cost kernels) is read from memory. A round scans its active rows
// with lane groups whose width follows the number of active rows: 4 lanes
// per row when most rows are active, 64 when a few rows scan long.
// The kernel does not need co-resident workgroups, so it can be captured in
// a HIP graph and replayed.
#include "cost_common.h"
#include "device_common.h"
#include "internal.h"

namespace prot {
namespace {

constexpr int kBatchThreads = 512;

template <int NMAX>
struct BatchShared {
    unsigned long long key[NMAX];  // (round << 32) | ~b of the column's current mate
    int32_t yb[NMAX];              // y(b)
    int32_t F[2][NMAX];            // free rows: this phase / next phase
    int32_t ab[2][NMAX];           // active rows of this round / the next
    int32_t ap[2][NMAX];           // their scan positions
    int32_t at[NMAX];              // column proposed to this round (-1: exhausted)
    int32_t L[NMAX];               // columns taken this phase
    uint16_t t[NMAX];              // -y(a)
    uint16_t skip[NMAX];           // phases row b is known to find nothing in
    long long red_k[kBatchThreads];
    double red_c[kBatchThreads];
    uint32_t nF[2], nact[2], nL, P, D;
    int32_t job;
    unsigned long long scanned;
};

// First admissible column not taken before round r, scanning row b from
// position pos with a group of GS lanes (all lanes of the group get the
// result). Keys and duals are in LDS.
// When the row is exhausted, *slack_out is the smallest k + t - need over the
// columns scanned if none of them was admissible, else 0.
template <int GS>
__device__ Hit group_scan(const int16_t *__restrict__ row, const uint16_t *t,
                          const unsigned long long *key, int n, int origin, int pos, int need,
                          uint32_t r0, uint32_t r, int gl, int gbase, int *slack_out)
{
    int mn = 0x7FFFFFFF;  // smallest k + t seen by this lane
    bool any_adm = false; // some scanned column was admissible (taken or not)
    constexpr int CH = GS * 8;
    constexpr int U = GS >= 16 ? 4 : 8;
    constexpr unsigned long long GM = GS == 64 ? ~0ull : ((1ull << GS) - 1ull);
    int lo[2], hi[2];
    const int c0 = origin + pos;
    if (c0 < n) {
        lo[0] = c0; hi[0] = n; lo[1] = 0; hi[1] = origin;
    } else {
        lo[0] = c0 - n; hi[0] = origin; lo[1] = 0; hi[1] = 0;
    }
    for (int sg = 0; sg < 2; ++sg) {
        const int slo = lo[sg], shi = hi[sg];
        if (slo >= shi) continue;
        int base = slo & ~7;
        int depth = 1;  // one chunk first: early rows usually hit in it
        while (base < shi) {
            uint4 kv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int col0 = base + u * CH + gl * 8;
                kv[u] = make_uint4(0u, 0u, 0u, 0u);
                if (u < depth && col0 < shi) kv[u] = *reinterpret_cast<const uint4 *>(row + col0);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (u >= depth) break;
                const int col0 = base + u * CH + gl * 8;
                uint32_t cand = 0;
                if (col0 < shi) {
                    const uint4 tv = *reinterpret_cast<const uint4 *>(t + col0);
                    const uint32_t rm = range_mask(col0, slo, shi);
                    cand = match_mask(kv[u], tv, need) & rm;
                    mn = min(mn, min_sum_masked(kv[u], tv, rm));
                }
                any_adm |= cand != 0u;
                uint32_t hit = 0;
                for (uint32_t c = cand; c; c &= c - 1) {
                    const int e = __builtin_ctz(c);
                    const uint32_t kr = (uint32_t)(key[col0 + e] >> 32);
                    if (!(kr >= r0 && kr < r)) hit |= 1u << e;
                }
                const unsigned long long bal = (__ballot(hit != 0u) >> gbase) & GM;
                if (bal) {
                    const int L = gbase + __builtin_ctzll(bal);
                    const uint32_t h = (uint32_t)__shfl((int)hit, L);
                    const int a = __shfl(col0, L) + __builtin_ctz(h);
                    return Hit{a >= origin ? a - origin : a - origin + n, a};
                }
            }
            base += depth * CH;
            depth = U;
        }
    }
#pragma unroll
    for (int off = GS / 2; off > 0; off >>= 1) mn = min(mn, __shfl_xor(mn, off));
    const bool adm = ((__ballot(any_adm) >> gbase) & GM) != 0ull;
    *slack_out = adm ? 0 : mn - need;
    return Hit{-1, -1};
}

// One proposal round over the active rows with groups of GS lanes.
template <int GS, int NMAX>
__device__ void round_pass(BatchShared<NMAX> &S, const int16_t *k, int64_t ldk, int n,
                           int origin_mode, uint32_t r0, uint32_t r, int ac, int nx)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int gl = lane & (GS - 1);
    const int gbase = lane - gl;
    const int g = tid / GS, ngroups = kBatchThreads / GS;
    const uint32_t nact = S.nact[ac];
    unsigned long long scanned = 0;
    for (uint32_t i = g; i < nact; i += ngroups) {
        const int b = S.ab[ac][i];
        const int pos = S.ap[ac][i];
        const int yb = S.yb[b];
        const int origin = origin_mode == 0 ? b : 0;
        Hit h{-1, -1};
        int slack = 0;
        const int skip = S.skip[b];
        if (skip == 0)
            h = group_scan<GS>(k + (int64_t)b * ldk, S.t, S.key, n, origin, pos, yb - 1, r0, r,
                               gl, gbase, &slack);
        if (gl != 0) continue;
        if (skip > 0) {
            // Exact fast-forward: an earlier full scan of this row found no
            // admissible column, every slack k + t - (y(b) - 1) was >= skip + 1
            // then, and since y(b) has grown by one per phase while t only
            // grows, no column can be admissible yet; the scan would exhaust.
            S.skip[b] = (uint16_t)(skip - 1);
        } else if (pos == 0 && slack >= 2) {
            // the row's first scan of this phase covered every column
            S.skip[b] = (uint16_t)min(slack - 1, 65535);
        }
        if (h.j >= 0) {
            scanned += (unsigned long long)(h.j - pos + 1);
            const unsigned long long kn = ((unsigned long long)r << 32) | (uint32_t)~(uint32_t)b;
            const unsigned long long old = atomicMax(&S.key[h.a], kn);
            S.at[i] = h.a;
            S.ap[ac][i] = h.j;
            atomicAdd(&S.P, 1u);
            if ((uint32_t)(old >> 32) < r) {
                // first proposal to a this round: a is in M' whoever wins;
                // step (II) evicts its old mate, (III a) will lower y(a)
                atomicAdd(&S.D, 1u);
                S.L[atomicAdd(&S.nL, 1u)] = h.a;
                if (old != 0ull) S.F[nx][atomicAdd(&S.nF[nx], 1u)] = (int32_t)~(uint32_t)old;
            }
        } else {
            // no admissible untaken column: b stays free in M', (III b)
            scanned += (unsigned long long)(n - pos);
            S.yb[b] = yb + 1;
            S.F[nx][atomicAdd(&S.nF[nx], 1u)] = b;
            S.at[i] = -1;
        }
    }
    if (scanned) atomicAdd(&S.scanned, scanned);
}

// Writes, in ascending order, the indices i < n with flag(i) into out;
// returns their number. All threads of the block call it.
template <int NMAX, class Flag>
__device__ int ordered_list(BatchShared<NMAX> &S, int n, Flag flag, int32_t *out)
{
    const int tid = threadIdx.x;
    const int per = (n + kBatchThreads - 1) / kBatchThreads;
    const int lo = min(n, tid * per), hi = min(n, lo + per);
    int c = 0;
    for (int i = lo; i < hi; ++i) c += flag(i) ? 1 : 0;
    long long *cnt = S.red_k;
    cnt[tid] = c;
    __syncthreads();
    for (int off = 1; off < kBatchThreads; off <<= 1) {
        const long long v = tid >= off ? cnt[tid - off] : 0;
        __syncthreads();
        cnt[tid] += v;
        __syncthreads();
    }
    int o = (int)cnt[tid] - c;
    for (int i = lo; i < hi; ++i)
        if (flag(i)) out[o++] = i;
    const int total = (int)cnt[kBatchThreads - 1];
    __syncthreads();
    return total;
}

template <int NMAX>
__device__ void solve_instance(const BatchArgs &A, int inst, BatchShared<NMAX> &S, bool timed)
{
    const int tid = threadIdx.x;
    const int n = A.n_arr[inst];
    const int64_t off = A.pt_off[inst];
    const int16_t *k = A.k + A.k_off[inst];
    const int64_t ldk = A.ldk_arr[inst];
    const int64_t T = (int64_t)floor(A.eps * (double)n + 1e-9);
    const int64_t bound = (2 * (int64_t)n * ((int64_t)floor(1.0 / A.eps) + 2) - n) / (T + 1);

    // Initial state (Section 2.2): y(b) = 1, y(a) = 0, M empty.
    for (int i = tid; i < n; i += kBatchThreads) {
        S.key[i] = 0ull;
        S.t[i] = 0;
        S.yb[i] = 1;
        S.F[0][i] = i;
        S.skip[i] = 0;
    }
    for (int i = n + tid; i < ((n + 7) & ~7); i += kBatchThreads) S.t[i] = 0;
    if (tid == 0) {
        S.nF[0] = (uint32_t)n;
        S.scanned = 0;
    }
    int64_t phases = 0, sum_free = 0, rounds = 0, max_rounds = 0;
    uint32_t r = 0;
    int cur = 0;
    int status = 0;
    __syncthreads();
    for (;;) {
        const uint32_t nF = S.nF[cur];
        if ((int64_t)nF <= T) break;
        if (A.max_phases > 0 && phases >= A.max_phases) {
            status = 1;
            break;
        }
        // watchdog: a cold start needs at most (2n(K + 2) - n) / (T + 1)
        // phases (Lemma 3.2 with eq. (4)); more means a fault
        if (phases >= bound) {
            status = -4;
            if (tid == 0)
                __hip_atomic_fetch_or(A.err, 256, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        phases += 1;
        sum_free += nF;
        const int nx = cur ^ 1;
        for (uint32_t i = tid; i < nF; i += kBatchThreads) {
            S.ab[0][i] = S.F[cur][i];
            S.ap[0][i] = 0;
        }
        __syncthreads();
        if (tid == 0) {
            S.nact[0] = nF;
            S.nF[nx] = 0;
            S.nL = 0;
        }
        const uint32_t r0 = r + 1;
        int ac = 0;
        int64_t phase_rounds = 0;
        for (;;) {
            r += 1;
            if (tid == 0) S.P = S.D = 0;
            __syncthreads();
            const uint32_t nact = S.nact[ac];
            const int64_t t_start = timed ? (int64_t)wall_clock64() : 0;
            // widest lane groups that still give every active row its own group
            if (nact > (uint32_t)kBatchThreads / 16)
                round_pass<4, NMAX>(S, k, ldk, n, A.origin, r0, r, ac, nx);
            else if (nact > (uint32_t)kBatchThreads / 64)
                round_pass<16, NMAX>(S, k, ldk, n, A.origin, r0, r, ac, nx);
            else
                round_pass<64, NMAX>(S, k, ldk, n, A.origin, r0, r, ac, nx);
            __syncthreads();
            if (timed && tid == 0 && 4u * r <= 3u * (uint32_t)kRoundTimeCap) {
                A.rtime[4 * (r - 1)] = t_start;
                A.rtime[4 * (r - 1) + 1] = (int64_t)wall_clock64();
                A.rtime[4 * (r - 1) + 2] = nact;
                A.rtime[4 * (r - 1) + 3] = phases;
            }
            const uint32_t P = S.P, D = S.D;
            if (P > 0) phase_rounds += 1;
            if (P == D) break;  // nobody lost a proposal: M' is maximal
            if (tid == 0) S.nact[ac ^ 1] = 0;
            __syncthreads();
            for (uint32_t i = tid; i < nact; i += kBatchThreads) {
                const int a = S.at[i];
                if (a < 0) continue;
                const int b = S.ab[ac][i];
                const unsigned long long kn = ((unsigned long long)r << 32) | (uint32_t)~(uint32_t)b;
                if (S.key[a] != kn) {  // lost: resume after the lost column
                    const uint32_t j = atomicAdd(&S.nact[ac ^ 1], 1u);
                    S.ab[ac ^ 1][j] = b;
                    S.ap[ac ^ 1][j] = S.ap[ac][i] + 1;
                }
            }
            ac ^= 1;
            __syncthreads();
        }
        rounds += phase_rounds;
        if (phase_rounds > max_rounds) max_rounds = phase_rounds;
        // Step (III a): y(a) -= 1 on every column of M'.
        const uint32_t nL = S.nL;
        for (uint32_t i = tid; i < nL; i += kBatchThreads) S.t[S.L[i]] += 1;
        cur = nx;
        __syncthreads();
    }
    const uint32_t nfree = S.nF[cur];

    // Matching from the keys; the free rows are F[cur], the free columns the
    // never-taken ones. Completion (Section 2.1): i-th free b (ascending)
    // with the i-th free a (ascending).
    int32_t *mb = S.ap[0], *ma = S.ap[1];
    for (int i = tid; i < n; i += kBatchThreads) {
        mb[i] = -1;
        S.at[i] = 0;
    }
    __syncthreads();
    for (int i = tid; i < n; i += kBatchThreads) {
        const unsigned long long kk = S.key[i];
        const int32_t b = kk ? (int32_t)~(uint32_t)kk : -1;
        ma[i] = b;
        if (b >= 0) mb[b] = i;
    }
    for (uint32_t i = tid; i < nfree; i += kBatchThreads) S.at[S.F[cur][i]] = 1;
    __syncthreads();
    if (A.complete && status >= 0) {
        const int nb = ordered_list(S, n, [&](int i) { return S.at[i] != 0; }, S.ab[0]);
        const int na = ordered_list(S, n, [&](int i) { return S.key[i] == 0ull; }, S.ab[1]);
        const int m = min(nb, na);
        for (int i = tid; i < m; i += kBatchThreads) {
            mb[S.ab[0][i]] = S.ab[1][i];
            ma[S.ab[1][i]] = S.ab[0][i];
        }
        __syncthreads();
    }

    // Outputs and per-instance statistics (fixed-order reductions).
    const float *X = A.X + off * A.d, *Y = A.Y + off * A.d;
    long long ks = 0;
    double cs = 0.0;
    for (int i = tid; i < n; i += kBatchThreads) {
        A.mate_a[off + i] = ma[i];
        A.mate_b[off + i] = mb[i];
        A.y_a[off + i] = -(int32_t)S.t[i];
        A.y_b[off + i] = S.yb[i];
        const int a = mb[i];
        if (a >= 0) {
            ks += k[(int64_t)i * ldk + a];
            double s = 0.0;
            for (int q = 0; q < A.d; ++q) {
                const double dq = __dsub_rn((double)X[(int64_t)i * A.d + q], (double)Y[(int64_t)a * A.d + q]);
                s = __dadd_rn(s, __dmul_rn(dq, dq));
            }
            cs = __dadd_rn(cs, s);
        }
    }
    S.red_k[tid] = ks;
    S.red_c[tid] = cs;
    __syncthreads();
    for (int o = kBatchThreads / 2; o > 0; o >>= 1) {
        if (tid < o) {
            S.red_k[tid] += S.red_k[tid + o];
            S.red_c[tid] = __dadd_rn(S.red_c[tid], S.red_c[tid + o]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        InstanceStats &st = A.stats[inst];
        const float m = A.m[inst];
        st.phases = phases;
        st.sum_free = sum_free;
        st.rounds = rounds;
        st.max_rounds = max_rounds;
        st.scanned = (int64_t)S.scanned;
        st.matched_in_phases = n - (int64_t)nfree;
        st.completed_pairs = A.complete ? (int64_t)nfree : 0;
        st.sum_k = S.red_k[0];
        st.threshold = T;
        st.status = status;
        st.kmax = m > 0.0f ? (int32_t)floor(1.0 / A.eps) : 0;
        st.cost_scale = (double)m;
        st.cost = m > 0.0f ? S.red_c[0] / (double)m : 0.0;
    }
    __syncthreads();
}

template <int NMAX>
__global__ void __launch_bounds__(kBatchThreads) batch_solve_kernel(BatchArgs A)
{
    __shared__ BatchShared<NMAX> S;
    for (;;) {
        if (threadIdx.x == 0)
            S.job = (int32_t)__hip_atomic_fetch_add(A.queue, 1u, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int job = S.job;
        __syncthreads();
        if (job >= A.batch) break;
        solve_instance<NMAX>(A, A.order[job], S, A.rtime != nullptr && job == 0);
    }
}

__global__ void batch_reset_kernel(unsigned int *queue) { *queue = 0u; }

}  // namespace

int32_t batch_max_n() { return 2048; }

hipError_t batch_grid(int32_t n_max, int32_t batch, int *grid)
{
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = n_max <= 1024
        ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_solve_kernel<1024>,
                                                       kBatchThreads, 0)
        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_solve_kernel<2048>,
                                                       kBatchThreads, 0);
    if (e != hipSuccess) return e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return e;
    int g = per_cu * cus;
    if (g > batch) g = batch;
    *grid = g < 1 ? 1 : g;
    return hipSuccess;
}

hipError_t launch_batch_solve(const BatchArgs &a, int32_t n_max, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(1), 0, s, a.queue);
    if (a.batch == 0) return hipGetLastError();
    if (n_max <= 1024)
        hipLaunchKernelGGL(batch_solve_kernel<1024>, dim3(grid), dim3(kBatchThreads), 0, s, a);
    else
        hipLaunchKernelGGL(batch_solve_kernel<2048>, dim3(grid), dim3(kBatchThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace prot
