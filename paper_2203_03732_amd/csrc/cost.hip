// Rounded-cost construction (arXiv:2203.03732, Section 2.1, eq. (1)).
//
// round_costs : a cost matrix already scaled to [0, 1] -> k = floor(c / eps),
//               the division in binary64. HBM-bound (4 B in, 2 B out).
// build_points: squared Euclidean costs of two point sets, scaled so the
//               largest is 1 (Section 1), then rounded. For the low
//               dimensions of the paper's synthetic workload (d = 2, 3) the
//               work is bound by the 2 B/entry write, so the distance is a
//               direct difference on the vector ALUs in binary32:
//               s = fma(x_j - y_j, x_j - y_j, s) in coordinate order.
//               k = floor((s / m) / eps) needs two binary64 divisions per
//               entry; instead, since that map is monotone in s, a small
//               table of the smallest binary32 s reaching each k is built
//               once per instance and each entry is classified against it,
//               which yields the identical integer.
#include "internal.h"

#include <float.h>
#include <math.h>

namespace prot {
namespace {

constexpr int kColsPerThread = 8;
constexpr int kBuildThreads = 256;
constexpr int kRowsPerBlock = 16;

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

__global__ void build_reset_kernel(Ctl *ctl)
{
    ctl->m = 0.0f;
    ctl->err = 0;
    ctl->kmax = 0;
}

template <int D>
__device__ inline float sqdist(const float *__restrict__ x, const float *__restrict__ y, int d)
{
    float s = 0.0f;
    if constexpr (D > 0) {
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const float t = __fsub_rn(x[j], y[j]);
            s = __fmaf_rn(t, t, s);
        }
    } else {
        for (int j = 0; j < d; ++j) {
            const float t = __fsub_rn(x[j], y[j]);
            s = __fmaf_rn(t, t, s);
        }
    }
    return s;
}

// Pass 1: m = max over all pairs of the binary32 squared distance. Block =
// 256 columns x kMaxRows rows; the rows' coordinates are staged in LDS.
constexpr int kMaxRows = 256;
constexpr int kMaxD = 16;   // coordinates staged per row (larger d: read from memory)

template <int D>
__global__ void __launch_bounds__(kBuildThreads)
points_max_kernel(const float *__restrict__ X, const float *__restrict__ Y, int64_t n,
                  int32_t d, Ctl *ctl)
{
    __shared__ float xs[kMaxRows * kMaxD];
    __shared__ float red[kBuildThreads / 64];
    const int64_t a = (int64_t)blockIdx.x * kBuildThreads + threadIdx.x;
    const int64_t b0 = (int64_t)blockIdx.y * kMaxRows;
    const int rows = (int)min<int64_t>(kMaxRows, n - b0);
    const bool staged = D > 0 || d <= kMaxD;
    const int dd = D > 0 ? D : d;
    if (staged)
        for (int i = threadIdx.x; i < rows * dd; i += kBuildThreads) xs[i] = X[b0 * dd + i];
    __syncthreads();
    float mx = 0.0f;
    bool bad = false;
    if (a < n) {
        const float *y = Y + a * dd;
        if (staged) {
            for (int r = 0; r < rows; ++r) {
                const float s = sqdist<D>(xs + r * dd, y, dd);
                bad |= !(s <= FLT_MAX);
                mx = fmaxf(mx, s);
            }
        } else {
            for (int r = 0; r < rows; ++r) {
                const float s = sqdist<D>(X + (b0 + r) * dd, y, dd);
                bad |= !(s <= FLT_MAX);
                mx = fmaxf(mx, s);
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        float m = red[0];
        for (int i = 1; i < kBuildThreads / 64; ++i) m = fmaxf(m, red[i]);
        // squared distances are >= 0, so their bit patterns order as floats do
        __hip_atomic_fetch_max(reinterpret_cast<unsigned *>(&ctl->m), __float_as_uint(m),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (bad) __hip_atomic_fetch_or(&ctl->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// k(s) = floor((s / m) / eps), both divisions binary64 (the definition).
__device__ inline double k_of(float s, double m, double eps)
{
    return floor(((double)s / m) / eps);
}

// th[j] = smallest binary32 s >= 0 with k(s) >= j, for j = 0..K; th[K+1] = +inf.
// k(s) is non-decreasing in s, and so in the bit pattern of s >= 0.
__global__ void thresholds_kernel(double eps, Ctl *ctl, float *th, int32_t kcap)
{
    const float mf = ctl->m;
    const double m = (double)mf;
    const int32_t K = (mf > 0.0f) ? (int32_t)floor(1.0 / eps) : 0;
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j == 0) ctl->kmax = K;
    if (j > K + 1 || j >= kcap) return;
    if (j == 0) { th[0] = 0.0f; return; }
    if (j == K + 1) { th[j] = __int_as_float(0x7f800000); return; }
    uint32_t lo = 0, hi = __float_as_uint(mf);  // k(m) = K >= j
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (k_of(__uint_as_float(mid), m, eps) >= (double)j) hi = mid; else lo = mid + 1;
    }
    th[j] = __uint_as_float(lo);
}

// k for one entry. v = s * inv in binary32 is within (K + 2) * 2^-22 of the
// exact s / (m eps) (inv and the product are each rounded once; the exact
// value is <= K + 1), and the binary64 definition is within 1e-10 of it. So
// when v is at least delta away from every integer, floor(v) is the
// definition's k; otherwise the threshold table decides.
__device__ inline int fast_k(float s, float inv, float delta, int K, bool &exact)
{
    const float v = __fmul_rn(s, inv);
    int g = (int)fminf(v, (float)K);
    g = g < 0 ? 0 : g;
    const float f = __fsub_rn(v, (float)g);
    exact = f >= delta && f <= 1.0f - delta && v < (float)K;
    return g;
}

__device__ inline int refine_k(float s, int g, int K, const float *__restrict__ th)
{
    while (g < K && s >= th[g + 1]) ++g;
    while (g > 0 && s < th[g]) --g;
    return g;
}

// Pass 2: k for every pair, 8 consecutive columns per thread (their points
// held in registers), kRowsPerBlock rows per block (coordinates in LDS);
// padding columns (n <= col < ldk) get 0x7FFF.
template <int D>
__global__ void __launch_bounds__(kBuildThreads)
points_k_kernel(const float *__restrict__ X, const float *__restrict__ Y, int64_t n,
                int32_t d, double eps, int16_t *__restrict__ k, int64_t ldk,
                const float *__restrict__ th, const Ctl *ctl)
{
    constexpr int DR = D > 0 ? D : 1;
    __shared__ float xs[kRowsPerBlock * kMaxD];
    const int64_t col0 = ((int64_t)blockIdx.x * kBuildThreads + threadIdx.x) * kColsPerThread;
    const int64_t b0 = (int64_t)blockIdx.y * kRowsPerBlock;
    const int rows = (int)min<int64_t>(kRowsPerBlock, n - b0);
    const int dd = D > 0 ? D : d;
    const bool staged = D > 0 || d <= kMaxD;
    if (staged)
        for (int i = threadIdx.x; i < rows * dd; i += kBuildThreads) xs[i] = X[b0 * dd + i];
    __syncthreads();
    if (col0 >= ldk) return;
    const float mf = ctl->m;
    const int32_t K = ctl->kmax;
    const float inv = (mf > 0.0f) ? (float)(1.0 / ((double)mf * eps)) : 0.0f;
    const float delta = (float)(K + 2) * 4.8e-7f;   // > (K + 2) * 2^-22 with margin
    float yv[kColsPerThread][DR];
#pragma unroll
    for (int e = 0; e < kColsPerThread; ++e)
#pragma unroll
        for (int j = 0; j < DR; ++j)
            yv[e][j] = (D > 0 && col0 + e < n) ? Y[(col0 + e) * DR + j] : 0.0f;
    for (int r = 0; r < rows; ++r) {
        const float *x = staged ? xs + r * dd : X + (b0 + r) * dd;
        float sv[kColsPerThread];
        int g[kColsPerThread];
        uint32_t slow = 0;
#pragma unroll
        for (int e = 0; e < kColsPerThread; ++e) {
            float s;
            if constexpr (D > 0) {
                s = 0.0f;
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const float t = __fsub_rn(x[j], yv[e][j]);
                    s = __fmaf_rn(t, t, s);
                }
            } else {
                s = col0 + e < n ? sqdist<0>(x, Y + (col0 + e) * dd, dd) : 0.0f;
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
        *reinterpret_cast<uint4 *>(k + (b0 + r) * ldk + col0) = w;
    }
}

}  // namespace

hipError_t launch_round_costs(const float *C, int64_t n, int64_t ldc, double eps,
                              int16_t *k, int64_t ldk, Ctl *ctl, hipStream_t s)
{
    hipLaunchKernelGGL(build_reset_kernel, dim3(1), dim3(1), 0, s, ctl);
    const int64_t per_block = (int64_t)kBuildThreads * kColsPerThread;
    dim3 grid((unsigned)((ldk + per_block - 1) / per_block), (unsigned)(n < 65535 ? n : 65535));
    if (n > 0)
        hipLaunchKernelGGL(round_costs_kernel, grid, dim3(kBuildThreads), 0, s, C, n, ldc,
                           eps, k, ldk, ctl);
    return hipGetLastError();
}

hipError_t launch_build_points(const float *X, const float *Y, int64_t n, int32_t d,
                               double eps, int16_t *k, int64_t ldk, float *m_out,
                               float *th, Ctl *ctl, hipStream_t s)
{
    hipLaunchKernelGGL(build_reset_kernel, dim3(1), dim3(1), 0, s, ctl);
    if (n == 0) return hipGetLastError();
    dim3 gmax((unsigned)((n + kBuildThreads - 1) / kBuildThreads),
              (unsigned)((n + kMaxRows - 1) / kMaxRows));
    if (d == 2)
        hipLaunchKernelGGL(points_max_kernel<2>, gmax, dim3(kBuildThreads), 0, s, X, Y, n, d, ctl);
    else if (d == 3)
        hipLaunchKernelGGL(points_max_kernel<3>, gmax, dim3(kBuildThreads), 0, s, X, Y, n, d, ctl);
    else
        hipLaunchKernelGGL(points_max_kernel<0>, gmax, dim3(kBuildThreads), 0, s, X, Y, n, d, ctl);
    const int32_t kcap = (int32_t)floor(1.0 / eps) + 2;
    hipLaunchKernelGGL(thresholds_kernel, dim3((kcap + 255) / 256), dim3(256), 0, s, eps, ctl,
                       th, kcap);
    const int64_t per_block = (int64_t)kBuildThreads * kColsPerThread;
    dim3 gk((unsigned)((ldk + per_block - 1) / per_block),
            (unsigned)((n + kRowsPerBlock - 1) / kRowsPerBlock));
    if (d == 2)
        hipLaunchKernelGGL(points_k_kernel<2>, gk, dim3(kBuildThreads), 0, s, X, Y, n, d, eps, k,
                           ldk, th, ctl);
    else if (d == 3)
        hipLaunchKernelGGL(points_k_kernel<3>, gk, dim3(kBuildThreads), 0, s, X, Y, n, d, eps, k,
                           ldk, th, ctl);
    else
        hipLaunchKernelGGL(points_k_kernel<0>, gk, dim3(kBuildThreads), 0, s, X, Y, n, d, eps, k,
                           ldk, th, ctl);
    if (m_out) {
        hipError_t e = hipMemcpyAsync(m_out, &ctl->m, sizeof(float), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

}  // namespace prot
