// Rounded-cost construction (arXiv:2203.03732, Section 2.1, eq. (1)).
//
// round_costs : a cost matrix already scaled to [0, 1] -> k = floor(c / eps),
//               the division in binary64. HBM-bound (4 B in, 2 B out).
// points      : squared Euclidean costs of point sets, scaled so the largest
//               is 1 (Section 1), then rounded; one instance or a batch of
//               independent instances (grid z = instance). The distance is a
//               direct difference on the vector ALUs in binary32,
//               s = fma(x_j - y_j, x_j - y_j, s) in coordinate order, so the
//               result is reproducible bit for bit. k = floor((s / m) / eps)
//               needs two binary64 divisions per entry; instead each entry is
//               classified by a binary32 product whose error is bounded, and
//               only entries within that bound of an integer are resolved
//               against a per-instance table of the smallest s reaching each
//               k (the map s -> k is monotone), giving the identical integer.
#include "cost_common.h"
#include "internal.h"

#include <float.h>
#include <math.h>

namespace prot {
namespace {

constexpr int kColsPerThread = 8;
constexpr int kBuildThreads = 256;
constexpr int kRowsPerBlock = 16;
constexpr int kMaxRows = 256;   // rows per block of the max pass
constexpr int kMaxD = 16;       // coordinates staged per row (larger d: read from memory)

__global__ void __launch_bounds__(kBuildThreads)
round_costs_kernel(const float *__restrict__ C, int64_t n, int64_t ldc, double eps,
                   int16_t *__restrict__ k, int64_t ldk, Ctl *ctl)
{
    const int64_t col0 = ((int64_t)blockIdx.x * kBuildThreads + threadIdx.x) * kColsPerThread;
    if (col0 >= ldk) return;
    bool bad = false;
    for (int64_t b = blockIdx.y; b < n; b += gridDim.y) {
        const float *crow = C + b * ldc;
        int16_t v[kColsPerThread];
#pragma unroll
        for (int e = 0; e < kColsPerThread; ++e) {
            const int64_t col = col0 + e;
            if (col < n) {
                const float c = crow[col];
                bad |= !(c >= 0.0f && c <= 1.0f);
                v[e] = (int16_t)floor((double)c / eps);
            } else {
                v[e] = 0x7FFF;
            }
        }
        uint4 w;
        w.x = (uint16_t)v[0] | ((uint32_t)(uint16_t)v[1] << 16);
        w.y = (uint16_t)v[2] | ((uint32_t)(uint16_t)v[3] << 16);
        w.z = (uint16_t)v[4] | ((uint32_t)(uint16_t)v[5] << 16);
        w.w = (uint16_t)v[6] | ((uint32_t)(uint16_t)v[7] << 16);
        *reinterpret_cast<uint4 *>(k + b * ldk + col0) = w;
    }
    if (bad) __hip_atomic_fetch_or(&ctl->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void build_reset_kernel(PointsJob j)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < j.batch; i += gridDim.x * blockDim.x)
        j.m[i] = 0.0f;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *j.err = 0;
        if (j.kmax_out) *j.kmax_out = 0;
    }
}

// Pass 1: m = max over all pairs of the binary32 squared distance. Block =
// 256 columns x kMaxRows rows of one instance; the rows' coordinates are
// staged in LDS.
template <int D>
__global__ void __launch_bounds__(kBuildThreads) points_max_kernel(PointsJob j)
{
    __shared__ float xs[kMaxRows * kMaxD];
    __shared__ float red[kBuildThreads / 64];
    const Instance in = j.instance(blockIdx.z);
    const int64_t a = (int64_t)blockIdx.x * kBuildThreads + threadIdx.x;
    const int64_t b0 = (int64_t)blockIdx.y * kMaxRows;
    if (b0 >= in.n || (int64_t)blockIdx.x * kBuildThreads >= in.n) return;
    const int rows = (int)min<int64_t>(kMaxRows, in.n - b0);
    const int dd = D > 0 ? D : j.d;
    const bool staged = D > 0 || j.d <= kMaxD;
    if (staged)
        for (int i = threadIdx.x; i < rows * dd; i += kBuildThreads) xs[i] = in.X[b0 * dd + i];
    __syncthreads();
    float mx = 0.0f;
    bool bad = false;
    if (a < in.n) {
        const float *y = in.Y + a * dd;
        for (int r = 0; r < rows; ++r) {
            const float s = sqdist<D>(staged ? xs + r * dd : in.X + (b0 + r) * dd, y, dd);
            bad |= !(s <= FLT_MAX);
            mx = fmaxf(mx, s);
        }
    }
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        float m = red[0];
        for (int i = 1; i < kBuildThreads / 64; ++i) m = fmaxf(m, red[i]);
        // squared distances are >= 0, so their bit patterns order as floats do
        __hip_atomic_fetch_max(reinterpret_cast<unsigned *>(&j.m[blockIdx.z]), __float_as_uint(m),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (bad) __hip_atomic_fetch_or(j.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// th[j] = smallest binary32 s >= 0 with k(s) >= j, for j = 0..K; th[K+1] = +inf.
__global__ void thresholds_kernel(PointsJob j)
{
    const float mf = j.m[blockIdx.z];
    const int32_t K = (mf > 0.0f) ? (int32_t)floor(1.0 / j.eps) : 0;
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && j.kmax_out && blockIdx.z == 0) *j.kmax_out = K;
    if (i > K + 1 || i >= j.kcap) return;
    j.th[(int64_t)blockIdx.z * j.kcap + i] = threshold_of(i, K, mf, j.eps);
}

// Pass 2: k for every pair, 8 consecutive columns per thread (their points
// held in registers), kRowsPerBlock rows per block (coordinates in LDS);
// padding columns (n <= col < ldk) get 0x7FFF.
template <int D>
__global__ void __launch_bounds__(kBuildThreads) points_k_kernel(PointsJob j)
{
    constexpr int DR = D > 0 ? D : 1;
    __shared__ float xs[kRowsPerBlock * kMaxD];
    const Instance in = j.instance(blockIdx.z);
    const int64_t col0 = ((int64_t)blockIdx.x * kBuildThreads + threadIdx.x) * kColsPerThread;
    const int64_t b0 = (int64_t)blockIdx.y * kRowsPerBlock;
    if (b0 >= in.n || (int64_t)blockIdx.x * kBuildThreads * kColsPerThread >= in.ldk) return;
    const int rows = (int)min<int64_t>(kRowsPerBlock, in.n - b0);
    const int dd = D > 0 ? D : j.d;
    const bool staged = D > 0 || j.d <= kMaxD;
    if (staged)
        for (int i = threadIdx.x; i < rows * dd; i += kBuildThreads) xs[i] = in.X[b0 * dd + i];
    __syncthreads();
    if (col0 >= in.ldk) return;
    const int64_t n = in.n;
    const float mf = j.m[blockIdx.z];
    const int32_t K = (mf > 0.0f) ? (int32_t)floor(1.0 / j.eps) : 0;
    const float inv = (mf > 0.0f) ? (float)(1.0 / ((double)mf * j.eps)) : 0.0f;
    const float delta = classify_margin(K);
    const float *th = j.th + (int64_t)blockIdx.z * j.kcap;
    float yv[kColsPerThread][DR];
#pragma unroll
    for (int e = 0; e < kColsPerThread; ++e)
#pragma unroll
        for (int q = 0; q < DR; ++q)
            yv[e][q] = (D > 0 && col0 + e < n) ? in.Y[(col0 + e) * DR + q] : 0.0f;
    for (int r = 0; r < rows; ++r) {
        const float *x = staged ? xs + r * dd : in.X + (b0 + r) * dd;
        float sv[kColsPerThread];
        int g[kColsPerThread];
        uint32_t slow = 0;
#pragma unroll
        for (int e = 0; e < kColsPerThread; ++e) {
            float s;
            if constexpr (D > 0) {
                s = 0.0f;
#pragma unroll
                for (int q = 0; q < D; ++q) {
                    const float t = __fsub_rn(x[q], yv[e][q]);
                    s = __fmaf_rn(t, t, s);
                }
            } else {
                s = col0 + e < n ? sqdist<0>(x, in.Y + (col0 + e) * dd, dd) : 0.0f;
            }
            bool ok;
            g[e] = fast_k(s, inv, delta, K, ok);
            sv[e] = s;
            slow |= (uint32_t)!ok << e;
        }
        if (slow) {
#pragma unroll
            for (int e = 0; e < kColsPerThread; ++e)
                if ((slow >> e) & 1u) g[e] = refine_k(sv[e], g[e], K, th);
        }
#pragma unroll
        for (int e = 0; e < kColsPerThread; ++e)
            if (col0 + e >= n) g[e] = 0x7FFF;
        uint4 w;
        w.x = (uint32_t)(uint16_t)g[0] | ((uint32_t)(uint16_t)g[1] << 16);
        w.y = (uint32_t)(uint16_t)g[2] | ((uint32_t)(uint16_t)g[3] << 16);
        w.z = (uint32_t)(uint16_t)g[4] | ((uint32_t)(uint16_t)g[5] << 16);
        w.w = (uint32_t)(uint16_t)g[6] | ((uint32_t)(uint16_t)g[7] << 16);
        *reinterpret_cast<uint4 *>(in.k + (b0 + r) * in.ldk + col0) = w;
    }
}

template <int D>
void launch_points_d(const PointsJob &j, int64_t n_max, int64_t ldk_max, hipStream_t s)
{
    dim3 gmax((unsigned)((n_max + kBuildThreads - 1) / kBuildThreads),
              (unsigned)((n_max + kMaxRows - 1) / kMaxRows), (unsigned)j.batch);
    hipLaunchKernelGGL(points_max_kernel<D>, gmax, dim3(kBuildThreads), 0, s, j);
    hipLaunchKernelGGL(thresholds_kernel, dim3((j.kcap + 255) / 256, 1, j.batch), dim3(256), 0,
                       s, j);
    const int64_t per_block = (int64_t)kBuildThreads * kColsPerThread;
    dim3 gk((unsigned)((ldk_max + per_block - 1) / per_block),
            (unsigned)((n_max + kRowsPerBlock - 1) / kRowsPerBlock), (unsigned)j.batch);
    hipLaunchKernelGGL(points_k_kernel<D>, gk, dim3(kBuildThreads), 0, s, j);
}

}  // namespace

hipError_t launch_round_costs(const float *C, int64_t n, int64_t ldc, double eps,
                              int16_t *k, int64_t ldk, Ctl *ctl, hipStream_t s)
{
    PointsJob j{};
    j.batch = 1;
    j.m = &ctl->m;
    j.err = &ctl->err;
    j.kmax_out = &ctl->kmax;
    hipLaunchKernelGGL(build_reset_kernel, dim3(1), dim3(64), 0, s, j);
    const int64_t per_block = (int64_t)kBuildThreads * kColsPerThread;
    dim3 grid((unsigned)((ldk + per_block - 1) / per_block), (unsigned)(n < 65535 ? n : 65535));
    if (n > 0)
        hipLaunchKernelGGL(round_costs_kernel, grid, dim3(kBuildThreads), 0, s, C, n, ldc,
                           eps, k, ldk, ctl);
    return hipGetLastError();
}

hipError_t launch_points(const PointsJob &j, int64_t n_max, int64_t ldk_max, hipStream_t s)
{
    hipLaunchKernelGGL(build_reset_kernel, dim3((j.batch + 255) / 256), dim3(256), 0, s, j);
    if (n_max == 0 || j.batch == 0) return hipGetLastError();
    if (j.d == 2) launch_points_d<2>(j, n_max, ldk_max, s);
    else if (j.d == 3) launch_points_d<3>(j, n_max, ldk_max, s);
    else launch_points_d<0>(j, n_max, ldk_max, s);
    return hipGetLastError();
}

}  // namespace prot
