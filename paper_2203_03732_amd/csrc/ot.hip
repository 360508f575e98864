// Optimal transport through unit copies (Section 4).
//
// The masses are scaled by theta = 4 max(n_b, n_a) / eps, supplies rounded
// down and demands rounded up into unit copies; the copies of one point are
// contiguous (point order). The phase loop runs on the copies (rows: supply
// copies, columns: demand copies) over an expanded cost matrix whose row p
// holds eq. (1) of supply point p against every demand copy; row b of the
// loop reads row rmap[b] = the point it copies, and a free copy's dual is
// raised to the largest dual of its point's copies. After the loop the
// matched copies give the plan (1/theta per pair), which is then made
// feasible: a demand point holding more than mu_a returns the excess (its
// edges in ascending b), and the mass still to be sent is paired with the
// room left at the demand points in index order (north-west corner rule on
// the running totals). Every binary64 operation that decides a plan entry is
// done in the same order as the definition, so the plan is bit-exact.
#include "internal.h"
#include "device_common.h"

#include <math.h>

namespace prot {
namespace {

constexpr int kScaleThreads = 1024;
constexpr int kStage = 2048;  // doubles staged through LDS by the ordered sums

// Block-wide exclusive prefix of v over the block's threads (all threads call).
__device__ long long block_exclusive(long long v, long long *tmp, long long *total)
{
    const int t = threadIdx.x;
    tmp[t] = v;
    __syncthreads();
    for (int off = 1; off < (int)blockDim.x; off <<= 1) {
        const long long add = t >= off ? tmp[t - off] : 0;
        __syncthreads();
        tmp[t] += add;
        __syncthreads();
    }
    const long long incl = tmp[t];
    if (total) *total = tmp[blockDim.x - 1];
    __syncthreads();
    return incl - v;
}

// Sum of p[0..n) in index order, by lane 0 of the block, staged through LDS
// (all threads call; the result is valid in thread 0).
__device__ double ordered_sum(const double *p, int64_t n, double *stage)
{
    double t = 0.0;
    for (int64_t base = 0; base < n; base += kStage) {
        const int m = (int)(n - base < kStage ? n - base : kStage);
        for (int i = threadIdx.x; i < m; i += blockDim.x) stage[i] = p[base + i];
        __syncthreads();
        if (threadIdx.x == 0)
            for (int i = 0; i < m; ++i) t += stage[i];
        __syncthreads();
    }
    return t;
}

// Running sums P[0] = 0, P[i+1] = P[i] + p[i] in index order (all threads call).
__device__ void ordered_prefix(const double *p, int64_t n, double *P, double *stage)
{
    __shared__ double carry;
    if (threadIdx.x == 0) {
        carry = 0.0;
        P[0] = 0.0;
    }
    __syncthreads();
    for (int64_t base = 0; base < n; base += kStage) {
        const int m = (int)(n - base < kStage ? n - base : kStage);
        for (int i = threadIdx.x; i < m; i += blockDim.x) stage[i] = p[base + i];
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = carry;
            for (int i = 0; i < m; ++i) {
                t += stage[i];
                stage[i] = t;
            }
            carry = t;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < m; i += blockDim.x) P[base + i + 1] = stage[i];
        __syncthreads();
    }
}

// Counts floor(theta nu_b) (down) or ceil(theta mu_a) (up) and their
// exclusive prefix off[0..n] (off[n] = total), one block.
__device__ long long copy_offsets(const double *m, int64_t n, double theta, bool up,
                                  int64_t *off, long long *tmp)
{
    const int64_t per = (n + blockDim.x - 1) / blockDim.x;
    const int64_t lo = threadIdx.x * per, hi = lo + per < n ? lo + per : n;
    long long mine = 0;
    for (int64_t i = lo; i < hi; ++i) {
        const double v = theta * m[i];
        mine += (long long)(up ? ceil(v) : floor(v));
    }
    __shared__ long long total;
    long long run = block_exclusive(mine, tmp, &total);
    for (int64_t i = lo; i < hi; ++i) {
        off[i] = run;
        const double v = theta * m[i];
        run += (long long)(up ? ceil(v) : floor(v));
    }
    if (threadIdx.x == 0) off[n] = total;
    __syncthreads();
    return total;
}

__global__ void __launch_bounds__(kScaleThreads)
ot_scale_kernel(const double *nu, int64_t n_b, const double *mu, int64_t n_a, double theta,
                int64_t *s_off, int64_t *d_off, OtInfo *info)
{
    __shared__ int bad;
    __shared__ long long tmp[kScaleThreads];
    __shared__ double stage[kStage];
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    // probability vectors: entries in [0, 1] (NaN fails), sums within 1e-9 of 1
    for (int64_t i = threadIdx.x; i < n_b; i += blockDim.x)
        if (!(nu[i] >= 0.0 && nu[i] <= 1.0)) atomicOr(&bad, 1);
    for (int64_t i = threadIdx.x; i < n_a; i += blockDim.x)
        if (!(mu[i] >= 0.0 && mu[i] <= 1.0)) atomicOr(&bad, 1);
    const double sb = ordered_sum(nu, n_b, stage);
    const double sa = ordered_sum(mu, n_a, stage);
    if (threadIdx.x == 0 && (fabs(sb - 1.0) > 1e-9 || fabs(sa - 1.0) > 1e-9)) atomicOr(&bad, 1);
    __syncthreads();
    if (bad) {
        if (threadIdx.x == 0) {
            info->err = 1;
            info->copies_b = info->copies_a = 0;
        }
        return;
    }
    const long long cb = copy_offsets(nu, n_b, theta, false, s_off, tmp);
    const long long ca = copy_offsets(mu, n_a, theta, true, d_off, tmp);
    if (threadIdx.x == 0) {
        info->copies_b = cb;
        info->copies_a = ca;
        info->err = (cb > ca || ca > 0x7FFFFFFFll) ? 2 : 0;
        info->repaired = 0.0;
    }
}

// owner[i] = the point whose copy range [off[p], off[p+1]) holds copy i.
__global__ void ot_owner_kernel(const int64_t *off, int64_t n_pts, int64_t copies, int32_t *owner)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < copies;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = n_pts - 1;  // largest p with off[p] <= i
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (off[mid] <= i) lo = mid;
            else hi = mid - 1;
        }
        owner[i] = (int32_t)lo;
    }
}

// Expanded rounded costs: k[p][j] = floor(C[p][col_pt[j]] / eps) (eq. (1),
// binary64), 0x7FFF past the last demand copy.
__global__ void ot_costs_kernel(const float *__restrict__ C, int64_t n_b, int64_t ldc,
                                const int32_t *__restrict__ col_pt, int64_t NA, double eps,
                                int16_t *__restrict__ k, int64_t ldk, Ctl *ctl)
{
    bool bad = false;
    for (int64_t p = blockIdx.y; p < n_b; p += gridDim.y) {
        for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < ldk;
             j += (int64_t)gridDim.x * blockDim.x) {
            int16_t v = 0x7FFF;
            if (j < NA) {
                const float c = C[p * ldc + col_pt[j]];
                bad |= !(c >= 0.0f && c <= 1.0f);
                v = (int16_t)floor((double)c / eps);
            }
            k[p * ldk + j] = v;
        }
    }
    if (__ballot(bad) && (threadIdx.x & 63) == 0)
        __hip_atomic_fetch_or(&ctl->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void ot_fill_kernel(int32_t *p, int64_t n, int32_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

constexpr int kPlanThreads = 256;

template <class T>
__device__ T block_sum(T v, T *sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = kPlanThreads / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    return sh[0];
}

// Pair counts per (supply point, demand point) and sum of k over the copies'
// matching (per-block partials in block order).
__global__ void __launch_bounds__(kPlanThreads) ot_count_kernel(OtPlanArgs a)
{
    __shared__ long long sk[kPlanThreads];
    long long mine = 0;
    for (int64_t b = blockIdx.x * (int64_t)kPlanThreads + threadIdx.x; b < a.NB;
         b += (int64_t)gridDim.x * kPlanThreads) {
        const int32_t c = a.mate_b[b];
        if (c < 0) continue;
        const int32_t p = a.row_pt[b], q = a.col_pt[c];
        atomicAdd(a.cnt + (int64_t)p * a.n_a + q, 1);
        mine += a.k[(int64_t)p * a.ldk + c];
    }
    const long long t = block_sum(mine, sk);
    if (threadIdx.x == 0) a.part_k[blockIdx.x] = t;
}

// One wave per demand point a: its column of the plan (1/theta per pair),
// the excess over mu_a returned in ascending b, and the room left q_a. The
// rows are read 64 at a time; only pairs with a nonzero count take part in
// the sequential binary64 steps, which the whole wave runs in ascending b
// (a zero entry gives nothing back and adding it leaves a sum unchanged), so
// every value equals the row-by-row definition's.
constexpr int kColWaves = 4;  // demand points per workgroup of ot_column_kernel
__global__ void __launch_bounds__(64 * kColWaves) ot_column_kernel(OtPlanArgs a)
{
    const int64_t q = blockIdx.x * (int64_t)kColWaves + threadIdx.x / 64;
    if (q >= a.n_a) return;  // the whole wave
    const int lane = threadIdx.x & 63;
    long long mine = 0;
    for (int64_t b0 = 0; b0 < a.n_b; b0 += 64)
        if (b0 + lane < a.n_b) mine += a.cnt[(b0 + lane) * a.n_a + q];
    for (int off = 32; off > 0; off >>= 1) mine += __shfl_xor(mine, off);
    double ex = (double)mine / a.theta - a.mu[q];
    double got = 0.0;
    for (int64_t b0 = 0; b0 < a.n_b; b0 += 64) {
        const int64_t b = b0 + lane;
        const int32_t c = b < a.n_b ? a.cnt[b * a.n_a + q] : 0;
        double mv = (double)c / a.theta;
        unsigned long long nz = __ballot(c != 0);
        while (nz) {
            const int l = __ffsll((long long)nz) - 1;
            nz &= nz - 1ull;
            double v = (double)__shfl(c, l) / a.theta;
            if (ex > 0.0) {
                const double take = v < ex ? v : ex;
                v = v - take;
                ex = ex - take;
            }
            got += v;
            if (lane == l) mv = v;
        }
        if (b < a.n_b) a.plan[b * a.ldp + q] = mv;
    }
    const double room = a.mu[q] - got;
    if (lane == 0) a.qv[q] = room > 0.0 ? room : 0.0;
}

// One wave per supply point b: what it still has to send (the row of the
// plan summed in ascending q over its nonzero entries, read 64 at a time).
__global__ void __launch_bounds__(64 * kColWaves) ot_row_kernel(OtPlanArgs a)
{
    const int64_t b = blockIdx.x * (int64_t)kColWaves + threadIdx.x / 64;
    if (b >= a.n_b) return;  // the whole wave
    const int lane = threadIdx.x & 63;
    double sent = 0.0;
    for (int64_t q0 = 0; q0 < a.n_a; q0 += 64) {
        const double v = q0 + lane < a.n_a ? a.plan[b * a.ldp + q0 + lane] : 0.0;
        unsigned long long nz = __ballot(v != 0.0);
        while (nz) {
            const int l = __ffsll((long long)nz) - 1;
            nz &= nz - 1ull;
            sent += __shfl(v, l);
        }
    }
    const double left = a.nu[b] - sent;
    if (lane == 0) a.rv[b] = left > 0.0 ? left : 0.0;
}

__global__ void __launch_bounds__(kScaleThreads) ot_prefix_kernel(OtPlanArgs a)
{
    __shared__ double stage[kStage];
    ordered_prefix(a.rv, a.n_b, a.R, stage);
    ordered_prefix(a.qv, a.n_a, a.Q, stage);
    if (threadIdx.x == 0) a.info->repaired = a.R[a.n_b];
}

// North-west corner on the running totals, then the plan's cost (per-block
// partials in block order).
__global__ void __launch_bounds__(kPlanThreads) ot_route_kernel(OtPlanArgs a)
{
    __shared__ double sc[kPlanThreads];
    double mine = 0.0;
    const int64_t total = a.n_b * a.n_a;
    for (int64_t e = blockIdx.x * (int64_t)kPlanThreads + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kPlanThreads) {
        const int64_t b = e / a.n_a, q = e - b * a.n_a;
        double v = a.plan[b * a.ldp + q];
        const double lo = a.R[b] > a.Q[q] ? a.R[b] : a.Q[q];
        const double hi = a.R[b + 1] < a.Q[q + 1] ? a.R[b + 1] : a.Q[q + 1];
        if (hi > lo) {
            v += hi - lo;
            a.plan[b * a.ldp + q] = v;
        }
        mine += v * (double)a.C[b * a.ldc + q];
    }
    const double t = block_sum(mine, sc);
    if (threadIdx.x == 0) a.part_c[blockIdx.x] = t;
}

// Per point: the smaller dual of its copies, and how many copies hold it (by
// Lemma 4.1 the others hold that value + 1; a wider spread sets err bit 16).
__global__ void ot_duals_kernel(const int32_t *y, const int64_t *off, int64_t n_pts, int32_t *lo,
                                int32_t *nlo, Ctl *ctl)
{
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n_pts;
         p += (int64_t)gridDim.x * blockDim.x) {
        int32_t mn = 0x7FFFFFFF, mx = -0x7FFFFFFF - 1, cnt = 0;
        for (int64_t i = off[p]; i < off[p + 1]; ++i) {
            const int32_t v = y[i];
            if (v < mn) {
                mn = v;
                cnt = 1;
            } else if (v == mn) {
                cnt += 1;
            }
            mx = v > mx ? v : mx;
        }
        if (off[p + 1] == off[p]) mn = 0;
        else if (mx - mn > 1)
            __hip_atomic_fetch_or(&ctl->err, 128, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        lo[p] = mn;
        nlo[p] = cnt;
    }
}

unsigned grid_of(int64_t n, int threads, unsigned cap = 65535u)
{
    const int64_t g = (n + threads - 1) / threads;
    return (unsigned)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

hipError_t launch_ot_scale(const double *nu, int64_t n_b, const double *mu, int64_t n_a,
                           double theta, int64_t *s_off, int64_t *d_off, OtInfo *info,
                           hipStream_t s)
{
    hipLaunchKernelGGL(ot_scale_kernel, dim3(1), dim3(kScaleThreads), 0, s, nu, n_b, mu, n_a,
                       theta, s_off, d_off, info);
    return hipGetLastError();
}

hipError_t launch_ot_prepare(const float *C, int64_t n_b, int64_t n_a, int64_t ldc, double eps,
                             const int64_t *s_off, int64_t NB, const int64_t *d_off, int64_t NA,
                             int32_t *row_pt, int32_t *col_pt, int16_t *k, int64_t ldk,
                             unsigned long long *ymax, Ctl *ctl, hipStream_t s)
{
    if (NB > 0)
        hipLaunchKernelGGL(ot_owner_kernel, dim3(grid_of(NB, 256)), dim3(256), 0, s, s_off, n_b,
                           NB, row_pt);
    if (NA > 0)
        hipLaunchKernelGGL(ot_owner_kernel, dim3(grid_of(NA, 256)), dim3(256), 0, s, d_off, n_a,
                           NA, col_pt);
    dim3 grid(grid_of(ldk, 256, 1024u), (unsigned)(n_b < 65535 ? n_b : 65535));
    hipLaunchKernelGGL(ot_costs_kernel, grid, dim3(256), 0, s, C, n_b, ldc, col_pt, NA, eps, k,
                       ldk, ctl);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // every copy starts at y(b) = 1, before the first phase
    return launch_fill_u64(ymax, n_b, 1ull, s);
}

hipError_t launch_ot_plan(const OtPlanArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(ot_fill_kernel, dim3(grid_of(a.n_b * a.n_a, 256, 4096u)), dim3(256), 0, s,
                       a.cnt, a.n_b * a.n_a, 0);
    hipLaunchKernelGGL(ot_count_kernel, dim3(kFinalizeBlocks), dim3(kPlanThreads), 0, s, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_ot_plan_finish(a, s);
}

hipError_t launch_ot_plan_finish(const OtPlanArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(ot_column_kernel, dim3(grid_of(a.n_a, kColWaves)), dim3(64 * kColWaves), 0,
                       s, a);
    hipLaunchKernelGGL(ot_row_kernel, dim3(grid_of(a.n_b, kColWaves)), dim3(64 * kColWaves), 0, s,
                       a);
    hipLaunchKernelGGL(ot_prefix_kernel, dim3(1), dim3(kScaleThreads), 0, s, a);
    hipLaunchKernelGGL(ot_route_kernel, dim3(kFinalizeBlocks), dim3(kPlanThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_ot_duals(const int32_t *y, const int64_t *off, int64_t n_pts, int32_t *lo,
                           int32_t *nlo, Ctl *ctl, hipStream_t s)
{
    hipLaunchKernelGGL(ot_duals_kernel, dim3(grid_of(n_pts, 64)), dim3(64), 0, s, y, off, n_pts,
                       lo, nlo, ctl);
    return hipGetLastError();
}

}  // namespace prot
