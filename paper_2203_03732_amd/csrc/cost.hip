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
#include "device_common.h"
#include "internal.h"

#include <algorithm>
#include <float.h>
#include <math.h>

namespace prot {
namespace {

constexpr int kColsPerThread = 8;
constexpr int kBuildThreads = 256;
constexpr int kRowsPerBlock = 16;
constexpr int kMaxRows = 256;   // rows per tile of the max pass
constexpr int kMaxCols = 1;     // columns per thread of the max pass
constexpr int kMaxD = 3;        // largest d of the low-dimensional kernels

// Eight rounded costs as bytes (uint8 matrix: every real entry is at most
// K <= 253; the padding sentinel 0x7FFF becomes 0xFF, still never admissible).
template <class T>
__device__ inline void store_k8(uint8_t *dst, const T *v)
{
    uint32_t b[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) b[e] = (uint32_t)v[e] > 255u ? 255u : (uint32_t)v[e];
    uint2 w;
    w.x = b[0] | (b[1] << 8) | (b[2] << 16) | (b[3] << 24);
    w.y = b[4] | (b[5] << 8) | (b[6] << 16) | (b[7] << 24);
    *reinterpret_cast<uint2 *>(dst) = w;
}

__global__ void __launch_bounds__(kBuildThreads)
round_costs_kernel(const float *__restrict__ C, int64_t n, int64_t na, int64_t ldc, double eps,
                   int16_t *__restrict__ k, int64_t ldk, Ctl *ctl, int k8)
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
            if (col < na) {
                const float c = crow[col];
                bad |= !(c >= 0.0f && c <= 1.0f);
                v[e] = (int16_t)floor((double)c / eps);
            } else {
                v[e] = 0x7FFF;
            }
        }
        if (k8) {
            store_k8(reinterpret_cast<uint8_t *>(k) + b * ldk + col0, v);
        } else {
            uint4 w;
            w.x = (uint16_t)v[0] | ((uint32_t)(uint16_t)v[1] << 16);
            w.y = (uint16_t)v[2] | ((uint32_t)(uint16_t)v[3] << 16);
            w.z = (uint16_t)v[4] | ((uint32_t)(uint16_t)v[5] << 16);
            w.w = (uint16_t)v[6] | ((uint32_t)(uint16_t)v[7] << 16);
            *reinterpret_cast<uint4 *>(k + b * ldk + col0) = w;
        }
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

// Low dimensions (d = 2, 3): the work is bound by the 2-byte writes of pass
// 2, so pairs are computed straight from registers and LDS.
// Pass 1: m = max over all pairs of the binary32 squared distance. Block =
// 256 x kMaxCols columns (kMaxCols consecutive ones per thread, so that each
// row read from LDS serves kMaxCols pairs) x tiles of kMaxRows rows of one
// instance (tile y, y + grid.y, ...); the rows' coordinates are staged in
// LDS. A batch combines the blocks'
// maxima with an atomic max per instance. One instance stores one maximum
// per block instead (thousands of atomics on one word queue up behind each
// other at the memory side) and the thresholds pass reduces them.
template <int D>
__global__ void __launch_bounds__(kBuildThreads) points_max_kernel(PointsJob j)
{
    static_assert(D > 0 && D <= kMaxD, "low-dimensional kernel");
    __shared__ float xs[kMaxRows * D];
    __shared__ float red[kBuildThreads / 64];
    const Instance in = j.instance(blockIdx.z);
    const int64_t a0 = ((int64_t)blockIdx.x * kBuildThreads + threadIdx.x) * kMaxCols;
    // A non-finite coordinate is caught where it is loaded; with finite
    // coordinates a distance can only overflow to +inf, which the maximum
    // keeps, so no per-pair test is needed. A missing column repeats the
    // thread's first one (a0 < na whenever any of its columns exists).
    bool bad = false;
    float mx = 0.0f;
    float y[kMaxCols][D];
    const bool col = a0 < in.na;
#pragma unroll
    for (int e = 0; e < kMaxCols; ++e) {
        const int64_t a = a0 + e < in.na ? a0 + e : a0;
#pragma unroll
        for (int q = 0; q < D; ++q) {
            y[e][q] = col ? in.Y[a * D + q] : 0.0f;
            bad |= !(fabsf(y[e][q]) <= FLT_MAX);
        }
    }
    if ((int64_t)blockIdx.x * kBuildThreads * kMaxCols < in.na) {
        for (int64_t b0 = (int64_t)blockIdx.y * kMaxRows; b0 < in.n;
             b0 += (int64_t)gridDim.y * kMaxRows) {
            const int rows = (int)min<int64_t>(kMaxRows, in.n - b0);
            __syncthreads();
            for (int i = threadIdx.x; i < rows * D; i += kBuildThreads) {
                const float v = in.X[b0 * D + i];
                bad |= !(fabsf(v) <= FLT_MAX);
                xs[i] = v;
            }
            __syncthreads();
            if (col)
                for (int r = 0; r < rows; ++r) {
                    float v[kMaxCols];
#pragma unroll
                    for (int e = 0; e < kMaxCols; ++e) v[e] = sqdist<D>(xs + r * D, y[e], D);
#pragma unroll
                    for (int e = 0; e < kMaxCols; ++e) mx = fmaxf(mx, v[e]);
                }
        }
        bad |= !(mx <= FLT_MAX);
    }
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    // one instance: a block that met a non-finite value stores -1 as its
    // maximum and the thresholds pass raises the error bit
    const bool block_bad = __syncthreads_or(bad) != 0;
    if (threadIdx.x == 0) {
        float m = red[0];
        for (int i = 1; i < kBuildThreads / 64; ++i) m = fmaxf(m, red[i]);
        if (j.mpart) {
            j.mpart[blockIdx.y * gridDim.x + blockIdx.x] = block_bad ? -1.0f : m;
        } else if (m > 0.0f) {
            // squared distances are >= 0, so their bit patterns order as floats do
            __hip_atomic_fetch_max(reinterpret_cast<unsigned *>(&j.m[blockIdx.z]),
                                   __float_as_uint(m), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    if (bad && !j.mpart) __hip_atomic_fetch_or(j.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Pruned exact maximum (one instance, d = 2, 3). The maximum of the binary32
// distances over all pairs is attained by a pair whose real distance is
// within a relative 2^-21 of it. (1) For each of the 2^d diagonal directions
// u, the point of X furthest along u and the point of Y furthest along -u;
// the largest binary32 distance among these pairs is a lower bound L <= m.
// (2) A point x can be in a pair of binary32 distance >= L only if the
// furthest corner of Y's bounding box is at real distance >= L (1 - 2^-21);
// that bound is evaluated in binary64 (exact differences and squares) and
// tested against L (1 - 1e-5); the same for y against X's box. (3) Every pair
// of surviving candidates is evaluated in binary32 and the maximum taken, so m
// is the maximum of the definition bit for bit; with no pruning possible (all
// pairs near the maximum) step 3 is the full n^2 pass.
__device__ inline uint32_t order_of(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float float_of(uint32_t o)
{
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o);
}

__global__ void prune_reset_kernel(PruneAux a)
{
    const int t = threadIdx.x;
    if (t < 16) a.ext[t] = 0ull;
    if (t < 12) a.bb[t] = ((t / 3) & 1) ? 0u : 0xFFFFFFFFu;  // min slots start high
    if (t < 2) a.cnt[t] = 0u;
}

template <int D>
__global__ void __launch_bounds__(256) extent_kernel(PointsJob j)
{
    constexpr int U = 1 << D;
    const PruneAux &P = j.prune;
    const int64_t n = j.n_single, na = j.na_single ? j.na_single : j.n_single;
    const int64_t top = n > na ? n : na;
    unsigned long long ex[U], ey[U];
    float lo[2][D], hi[2][D];
#pragma unroll
    for (int u = 0; u < U; ++u) ex[u] = ey[u] = 0ull;
#pragma unroll
    for (int q = 0; q < D; ++q) {
        lo[0][q] = lo[1][q] = FLT_MAX;
        hi[0][q] = hi[1][q] = -FLT_MAX;
    }
    bool bad = false;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < top;
         i += (int64_t)gridDim.x * blockDim.x) {
        const bool hx = i < n, hy = i < na;
        float x[D], y[D];
#pragma unroll
        for (int q = 0; q < D; ++q) {
            x[q] = hx ? j.X[i * D + q] : 0.0f;
            y[q] = hy ? j.Y[i * D + q] : 0.0f;
            bad |= !(fabsf(x[q]) <= FLT_MAX) || !(fabsf(y[q]) <= FLT_MAX);
            if (hx) {
                lo[0][q] = fminf(lo[0][q], x[q]);
                hi[0][q] = fmaxf(hi[0][q], x[q]);
            }
            if (hy) {
                lo[1][q] = fminf(lo[1][q], y[q]);
                hi[1][q] = fmaxf(hi[1][q], y[q]);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            float px = 0.0f, py = 0.0f;
#pragma unroll
            for (int q = 0; q < D; ++q) {
                px += ((u >> q) & 1) ? x[q] : -x[q];
                py += ((u >> q) & 1) ? -y[q] : y[q];
            }
            const unsigned long long kx = ((unsigned long long)order_of(px) << 32) | (uint32_t)i;
            const unsigned long long ky = ((unsigned long long)order_of(py) << 32) | (uint32_t)i;
            if (hx) ex[u] = kx > ex[u] ? kx : ex[u];
            if (hy) ey[u] = ky > ey[u] ? ky : ey[u];
        }
    }
    // wave reductions, then one atomic per wave
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const unsigned long long ox = __shfl_xor(ex[u], off), oy = __shfl_xor(ey[u], off);
            ex[u] = ox > ex[u] ? ox : ex[u];
            ey[u] = oy > ey[u] ? oy : ey[u];
        }
#pragma unroll
        for (int q = 0; q < D; ++q)
#pragma unroll
            for (int w = 0; w < 2; ++w) {
                lo[w][q] = fminf(lo[w][q], __shfl_xor(lo[w][q], off));
                hi[w][q] = fmaxf(hi[w][q], __shfl_xor(hi[w][q], off));
            }
    }
    // then over the block's four waves in LDS, and one set of atomics per
    // block (all waves updating the same few words would serialise on them)
    __shared__ unsigned long long s_ex[4][U], s_ey[4][U];
    __shared__ float s_lo[4][2][D], s_hi[4][2][D];
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            s_ex[wv][u] = ex[u];
            s_ey[wv][u] = ey[u];
        }
#pragma unroll
        for (int q = 0; q < D; ++q)
#pragma unroll
            for (int w = 0; w < 2; ++w) {
                s_lo[wv][w][q] = lo[w][q];
                s_hi[wv][w][q] = hi[w][q];
            }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int v = 1; v < (int)(blockDim.x >> 6); ++v) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                ex[u] = s_ex[v][u] > ex[u] ? s_ex[v][u] : ex[u];
                ey[u] = s_ey[v][u] > ey[u] ? s_ey[v][u] : ey[u];
            }
#pragma unroll
            for (int q = 0; q < D; ++q)
#pragma unroll
                for (int w = 0; w < 2; ++w) {
                    lo[w][q] = fminf(lo[w][q], s_lo[v][w][q]);
                    hi[w][q] = fmaxf(hi[w][q], s_hi[v][w][q]);
                }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            __hip_atomic_fetch_max(&P.ext[u], ex[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_max(&P.ext[8 + u], ey[u], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
#pragma unroll
        for (int q = 0; q < D; ++q)
#pragma unroll
            for (int w = 0; w < 2; ++w) {
                __hip_atomic_fetch_min(&P.bb[6 * w + q], order_of(lo[w][q]), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_max(&P.bb[6 * w + 3 + q], order_of(hi[w][q]), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
    }
    if (bad) __hip_atomic_fetch_or(j.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int D>
__device__ inline float prune_lower_bound(const PointsJob &j)
{
    // the largest binary32 distance among the directional extreme points
    constexpr int U = 1 << D;
    const PruneAux &P = j.prune;
    float L = 0.0f;
    for (int u1 = 0; u1 < U; ++u1)
        for (int u2 = 0; u2 < U; ++u2) {
            const int64_t bi = (int64_t)(uint32_t)P.ext[u1], ai = (int64_t)(uint32_t)P.ext[8 + u2];
            L = fmaxf(L, sqdist<D>(j.X + bi * D, j.Y + ai * D, D));
        }
    return L;
}

template <int D>
__global__ void __launch_bounds__(256) prune_kernel(PointsJob j)
{
    const PruneAux &P = j.prune;
    const int64_t n = j.n_single, na = j.na_single ? j.na_single : j.n_single;
    const int64_t top = n > na ? n : na;
    const double L = (double)prune_lower_bound<D>(j) * (1.0 - 1e-5);
    double blo[2][D], bhi[2][D];
#pragma unroll
    for (int q = 0; q < D; ++q)
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            blo[w][q] = (double)float_of(P.bb[6 * w + q]);
            bhi[w][q] = (double)float_of(P.bb[6 * w + 3 + q]);
        }
    const int lane = threadIdx.x & 63;
    for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < top;
         base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = base + threadIdx.x;
        bool cx = false, cy = false;
        if (i < top) {
            // furthest corner of the other set's box, per coordinate
            double ux = 0.0, uy = 0.0;
#pragma unroll
            for (int q = 0; q < D; ++q) {
                const double x = i < n ? (double)j.X[i * D + q] : 0.0;
                const double y = i < na ? (double)j.Y[i * D + q] : 0.0;
                const double a0 = x - blo[1][q], a1 = x - bhi[1][q];
                const double b0 = y - blo[0][q], b1 = y - bhi[0][q];
                ux += fmax(a0 * a0, a1 * a1);
                uy += fmax(b0 * b0, b1 * b1);
            }
            cx = i < n && ux >= L;
            cy = i < na && uy >= L;
        }
        const unsigned long long bx = __ballot(cx), by = __ballot(cy);
        uint32_t ox = 0, oy = 0;
        if (lane == 0) {
            if (bx) ox = atomicAdd(&P.cnt[0], (uint32_t)__popcll(bx));
            if (by) oy = atomicAdd(&P.cnt[1], (uint32_t)__popcll(by));
        }
        ox = __builtin_amdgcn_readfirstlane(ox);
        oy = __builtin_amdgcn_readfirstlane(oy);
        if (cx) P.cx[ox + lanes_below(bx)] = (int32_t)i;
        if (cy) P.cy[oy + lanes_below(by)] = (int32_t)i;
    }
}

// Every candidate pair: tiles of kMaxRows x-candidates (staged in LDS) by 256
// y-candidates, visited by a fixed grid.
template <int D>
__global__ void __launch_bounds__(kBuildThreads) pairs_max_kernel(PointsJob j)
{
    __shared__ float xs[kMaxRows * D];
    __shared__ float red[kBuildThreads / 64];
    const PruneAux &P = j.prune;
    const int64_t nx = P.cnt[0], ny = P.cnt[1];
    const int64_t tx = (nx + kMaxRows - 1) / kMaxRows, ty = (ny + kBuildThreads - 1) / kBuildThreads;
    float mx = 0.0f;
    for (int64_t t = blockIdx.x; t < tx * ty; t += gridDim.x) {
        const int64_t r0 = (t / ty) * kMaxRows, c = (t % ty) * kBuildThreads + threadIdx.x;
        const int rows = (int)min<int64_t>(kMaxRows, nx - r0);
        __syncthreads();
        for (int i = threadIdx.x; i < rows * D; i += kBuildThreads)
            xs[i] = j.X[(int64_t)P.cx[r0 + i / D] * D + i % D];
        __syncthreads();
        if (c < ny) {
            float y[D];
            const int64_t a = P.cy[c];
#pragma unroll
            for (int q = 0; q < D; ++q) y[q] = j.Y[a * D + q];
            for (int r = 0; r < rows; ++r) mx = fmaxf(mx, sqdist<D>(xs + r * D, y, D));
        }
    }
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        float m = red[0];
        for (int i = 1; i < kBuildThreads / 64; ++i) m = fmaxf(m, red[i]);
        if (!(m <= FLT_MAX))
            __hip_atomic_fetch_or(j.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (j.mpart)
            j.mpart[blockIdx.x] = m;
        else if (m > 0.0f)
            __hip_atomic_fetch_max(reinterpret_cast<unsigned *>(j.m), __float_as_uint(m),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// threshold_of by one wave: the same smallest bit pattern, found by a
// 64-way search. Invariant: the answer lies in [lo, hi] and k(hi) >= j. Each
// step probes lo + step*(l+1) on lane l; as k is non-decreasing in the bit
// pattern, the lanes whose probe reaches j form a suffix, and the answer lies
// just past the last probe that does not. About 6 dependent steps instead of
// the 30 of a binary search, each with the same binary64 evaluation.
__device__ inline float threshold_wave(int32_t j, int32_t K, float mf, double eps, int metric)
{
    if (j == 0) return 0.0f;
    if (j > K) return __int_as_float(0x7f800000);
    const double m = (double)mf;
    const uint32_t lane = threadIdx.x & 63u;
    uint32_t lo = 0, hi = __float_as_uint(mf);
    while (hi - lo >= 64u) {
        const uint32_t step = (hi - lo) / 64u;
        const uint32_t p = lo + step * (lane + 1u);  // lane 63: lo + 64 step <= hi
        const unsigned long long hit =
            __ballot(k_of(__uint_as_float(p), m, eps, metric) >= (double)j);
        if (hit) {
            const uint32_t f = (uint32_t)__ffsll((long long)hit) - 1u;
            hi = lo + step * (f + 1u);
            if (f) lo += step * f + 1u;
        } else {
            lo += step * 64u + 1u;
        }
    }
    // at most 64 candidates left, lo .. hi, one per lane; k(hi) >= j
    const uint32_t p = lo + lane;
    const unsigned long long hit =
        __ballot(p <= hi && k_of(__uint_as_float(p), m, eps, metric) >= (double)j);
    return __uint_as_float(hit ? lo + (uint32_t)__ffsll((long long)hit) - 1u : hi);
}

constexpr int kThresholdBlocks = 256;  // at most, per instance (4 thresholds a block at a time)

// th[j] = smallest binary32 s >= 0 with k(s) >= j, for j = 0..K; th[K+1] = +inf.
// One wave per threshold.
// With per-block maxima (one instance) every block first reduces them to m;
// block 0 stores m for the later passes and, when the plain maximum pass
// produced them (nmpart_err), sets the error word: bit 0 if a block met a
// non-finite value, every other bit cleared for the solve that follows.
__global__ void thresholds_kernel(PointsJob j)
{
    float mf;
    if (j.mpart) {
        __shared__ float red[4];
        float v = 0.0f;
        bool bad = false;
        for (int i = threadIdx.x; i < j.nmpart; i += blockDim.x) {
            const float x = j.mpart[i];
            bad |= x < 0.0f;
            v = fmaxf(v, x);
        }
        for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
        const bool any_bad = __syncthreads_or(bad) != 0;
        mf = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            j.m[0] = mf;
            if (j.nmpart_err) *j.err = any_bad ? 1 : 0;
        }
    } else {
        mf = j.m[blockIdx.z];
    }
    const int32_t K = (mf > 0.0f) ? (int32_t)floor(1.0 / j.eps) : 0;
    if (blockIdx.x == 0 && threadIdx.x == 0 && j.kmax_out && blockIdx.z == 0) *j.kmax_out = K;
    const int32_t waves = (int32_t)(gridDim.x * (blockDim.x / 64u));
    for (int32_t i = (int32_t)(blockIdx.x * (blockDim.x / 64u) + threadIdx.x / 64u);
         i <= K + 1 && i < j.kcap; i += waves) {
        const float v = threshold_wave(i, K, mf, j.eps, j.metric);
        if ((threadIdx.x & 63u) == 0) j.th[(int64_t)blockIdx.z * j.kcap + i] = v;
    }
}

inline unsigned threshold_blocks(int32_t kcap)
{
    return (unsigned)std::min(kThresholdBlocks, (kcap + 3) / 4);
}

// Pass 2: k for every pair, 8 consecutive columns per thread (their points
// held in registers), kRowsPerBlock rows per block (coordinates in LDS);
// padding columns (n <= col < ldk) get 0x7FFF.
template <int D>
__global__ void __launch_bounds__(kBuildThreads) points_k_kernel(PointsJob j)
{
    static_assert(D > 0 && D <= kMaxD, "low-dimensional kernel");
    __shared__ float xs[kRowsPerBlock * D];
    const Instance in = j.instance(blockIdx.z);
    const int64_t col0 = ((int64_t)blockIdx.x * kBuildThreads + threadIdx.x) * kColsPerThread;
    const int64_t b0 = (int64_t)blockIdx.y * kRowsPerBlock;
    if (b0 >= in.n || (int64_t)blockIdx.x * kBuildThreads * kColsPerThread >= in.ldk) return;
    const int rows = (int)min<int64_t>(kRowsPerBlock, in.n - b0);
    for (int i = threadIdx.x; i < rows * D; i += kBuildThreads) xs[i] = in.X[b0 * D + i];
    __syncthreads();
    if (col0 >= in.ldk) return;
    const int64_t n = in.na;  // columns
    const float mf = j.m[blockIdx.z];
    const int32_t K = (mf > 0.0f) ? (int32_t)floor(1.0 / j.eps) : 0;
    // Euclidean: an estimate from sqrt(s), made exact by the threshold table
    const bool euclid = j.metric == 1;
    const float inv = (mf > 0.0f) ? (float)(1.0 / ((euclid ? sqrt((double)mf) : (double)mf) *
                                                     j.eps))
                                  : 0.0f;
    const float delta = classify_margin(K);
    const float *th = j.th + (int64_t)blockIdx.z * j.kcap;
    float yv[kColsPerThread][D];
#pragma unroll
    for (int e = 0; e < kColsPerThread; ++e)
#pragma unroll
        for (int q = 0; q < D; ++q) yv[e][q] = col0 + e < n ? in.Y[(col0 + e) * D + q] : 0.0f;
    uint32_t pad = 0;  // padding columns of this thread
#pragma unroll
    for (int e = 0; e < kColsPerThread; ++e) pad |= (uint32_t)(col0 + e >= n) << e;
    for (int r = 0; r < rows; ++r) {
        const float *x = xs + r * D;
        float sv[kColsPerThread];
        int g[kColsPerThread];
        bool all_ok = true;
#pragma unroll
        for (int e = 0; e < kColsPerThread; ++e) {
            const float s = sqdist<D>(x, yv[e], D);
            bool ok;
            if (euclid) {
                g[e] = (int)__fmul_rn(__fsqrt_rn(s), inv);
                ok = false;
            } else {
                g[e] = fast_k(s, inv, delta, K, ok);
            }
            sv[e] = s;
            all_ok &= ok;
        }
        if (!all_ok) {
            // rare (squared cost): entries within the margin of a rounding
            // boundary; Euclidean: every entry
#pragma unroll
            for (int e = 0; e < kColsPerThread; ++e) {
                bool ok = false;
                if (!euclid) fast_k(sv[e], inv, delta, K, ok);
                if (!ok) g[e] = refine_k(sv[e], g[e], K, th);
            }
        }
        if (pad) {
#pragma unroll
            for (int e = 0; e < kColsPerThread; ++e)
                if ((pad >> e) & 1u) g[e] = 0x7FFF;
        }
        if (j.k8) {
            store_k8(reinterpret_cast<uint8_t *>(in.k) + (b0 + r) * in.ldk + col0, g);
        } else {
            uint4 w;
            w.x = (uint32_t)(uint16_t)g[0] | ((uint32_t)(uint16_t)g[1] << 16);
            w.y = (uint32_t)(uint16_t)g[2] | ((uint32_t)(uint16_t)g[3] << 16);
            w.z = (uint32_t)(uint16_t)g[4] | ((uint32_t)(uint16_t)g[5] << 16);
            w.w = (uint32_t)(uint16_t)g[6] | ((uint32_t)(uint16_t)g[7] << 16);
            *reinterpret_cast<uint4 *>(in.k + (b0 + r) * in.ldk + col0) = w;
        }
    }
}

// General d: a 64 x 64 block of pairs, 4 x 4 pairs per thread, coordinates
// staged through LDS 16 at a time (coordinate-major, so each thread reads its
// 4 rows and its 4 columns with one 16-byte LDS load each). Every pair still
// accumulates fma(x_j - y_j, x_j - y_j, s) in coordinate order; coordinates
// past d are staged as 0 and add exactly nothing. PASS 0 takes the maximum,
// PASS 1 writes the rounded costs.
constexpr int kTile = 64;
constexpr int kTj = 16;

template <int PASS, bool L1 = false>
__global__ void __launch_bounds__(256) points_tile_kernel(PointsJob j)
{
    __shared__ __align__(16) float xs[kTj][kTile + 4];
    __shared__ __align__(16) float ys[kTj][kTile + 4];
    __shared__ float red[4];
    const Instance in = j.instance(blockIdx.z);
    const int64_t n = in.n, na = in.na;  // rows, columns
    const int64_t b0 = (int64_t)blockIdx.y * kTile, a0 = (int64_t)blockIdx.x * kTile;
    if (b0 >= n || a0 >= (PASS ? in.ldk : na)) return;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int d = j.d;
    float acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[i][c] = 0.0f;
    for (int j0 = 0; j0 < d; j0 += kTj) {
        for (int q = tid; q < kTile * kTj; q += 256) {
            const int r = q / kTj, jj = q - r * kTj;
            const bool cj = j0 + jj < d;
            xs[jj][r] = (cj && b0 + r < n) ? in.X[(b0 + r) * d + j0 + jj] : 0.0f;
            ys[jj][r] = (cj && a0 + r < na) ? in.Y[(a0 + r) * d + j0 + jj] : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int jj = 0; jj < kTj; ++jj) {
            const float4 xv = *reinterpret_cast<const float4 *>(&xs[jj][ty * 4]);
            const float4 yv = *reinterpret_cast<const float4 *>(&ys[jj][tx * 4]);
            const float xr[4] = {xv.x, xv.y, xv.z, xv.w};
            const float yc[4] = {yv.x, yv.y, yv.z, yv.w};
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const float t = __fsub_rn(xr[i], yc[c]);
                    if constexpr (L1) acc[i][c] = __fadd_rn(acc[i][c], fabsf(t));
                    else acc[i][c] = __fmaf_rn(t, t, acc[i][c]);
                }
        }
        __syncthreads();
    }
    if constexpr (PASS == 0) {
        float mx = 0.0f;
        bool bad = false;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (b0 + ty * 4 + i < n && a0 + tx * 4 + c < na) {
                    bad |= !(acc[i][c] <= FLT_MAX);
                    mx = fmaxf(mx, acc[i][c]);
                }
        for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
        if ((tid & 63) == 0) red[tid >> 6] = mx;
        __syncthreads();
        if (tid == 0) {
            const float m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
            __hip_atomic_fetch_max(reinterpret_cast<unsigned *>(&j.m[blockIdx.z]),
                                   __float_as_uint(m), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        if (bad) __hip_atomic_fetch_or(j.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        const float mf = j.m[blockIdx.z];
        const int32_t K = (mf > 0.0f) ? (int32_t)floor(1.0 / j.eps) : 0;
        const bool euclid = j.metric == 1;
        const float inv = (mf > 0.0f) ? (float)(1.0 / ((euclid ? sqrt((double)mf) : (double)mf) *
                                                         j.eps))
                                      : 0.0f;
        const float delta = classify_margin(K);
        const float *th = j.th + (int64_t)blockIdx.z * j.kcap;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t row = b0 + ty * 4 + i;
            if (row >= n) continue;
            int g[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int64_t col = a0 + tx * 4 + c;
                if (col >= na) {
                    g[c] = 0x7FFF;
                    continue;
                }
                if constexpr (L1) {
                    // half the L1 distance, clamped to 1, eq. (1) in binary64
                    g[c] = (int)floor(fmin((double)acc[i][c] * 0.5, 1.0) / j.eps);
                } else if (euclid) {
                    g[c] = refine_k(acc[i][c], (int)__fmul_rn(__fsqrt_rn(acc[i][c]), inv), K,
                                    th);
                } else {
                    bool ok;
                    g[c] = fast_k(acc[i][c], inv, delta, K, ok);
                    if (!ok) g[c] = refine_k(acc[i][c], g[c], K, th);
                }
            }
            if (j.k8) {
                uint32_t q[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) q[c] = (uint32_t)g[c] > 255u ? 255u : (uint32_t)g[c];
                *reinterpret_cast<uint32_t *>(reinterpret_cast<uint8_t *>(in.k) + row * in.ldk + a0 +
                                              tx * 4) = q[0] | (q[1] << 8) | (q[2] << 16) | (q[3] << 24);
            } else {
                uint2 w;
                w.x = (uint32_t)(uint16_t)g[0] | ((uint32_t)(uint16_t)g[1] << 16);
                w.y = (uint32_t)(uint16_t)g[2] | ((uint32_t)(uint16_t)g[3] << 16);
                *reinterpret_cast<uint2 *>(in.k + row * in.ldk + a0 + tx * 4) = w;
            }
        }
    }
}

// Section 5's image cost: each vector divided by its sum (binary32, the sum
// taken in coordinate order by one lane). kNormFloats coordinates of a block's
// vectors are staged in LDS. Entries must be finite and nonnegative with a
// positive finite sum (err bit 1 otherwise). Block 0 also records the cost
// scale 2 (the L1 distance of two such vectors is at most 2) and K.
constexpr int kNormFloats = 12288;

__global__ void __launch_bounds__(256) l1_normalize_kernel(PointsJob j, const float *src,
                                                           int64_t n, float *dst)
{
    __shared__ float v[kNormFloats];
    __shared__ float sums[64];
    __shared__ int bad;
    const int d = j.d;
    const int per = min(64, kNormFloats / d);
    const int64_t first = (int64_t)blockIdx.x * per;
    if (first >= n) return;
    const int cnt = (int)min<int64_t>(per, n - first);
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < cnt * d; i += blockDim.x) {
        const float x = src[first * d + i];
        if (!(x >= 0.0f && x <= FLT_MAX)) bad = 1;
        v[i] = x;
    }
    __syncthreads();
    if ((int)threadIdx.x < cnt) {
        float t = 0.0f;
        for (int q = 0; q < d; ++q) t = __fadd_rn(t, v[threadIdx.x * d + q]);
        if (!(t > 0.0f && t <= FLT_MAX)) bad = 1;
        sums[threadIdx.x] = t;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < cnt * d; i += blockDim.x)
        dst[first * d + i] = __fdiv_rn(v[i], sums[i / d]);
    if (threadIdx.x == 0) {
        if (bad) __hip_atomic_fetch_or(j.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (blockIdx.x == 0) {
            j.m[0] = 2.0f;
            if (j.kmax_out) *j.kmax_out = (int32_t)floor(1.0 / j.eps);
        }
    }
}

void launch_points_l1(const PointsJob &j, int64_t n_max, int64_t ldk_max, hipStream_t s)
{
    // one instance (the batched solver keeps the squared cost)
    const int64_t nb = j.n_single, na = j.na_single ? j.na_single : j.n_single;
    const int per = std::min(64, kNormFloats / j.d);
    PointsJob jn = j;
    jn.X = j.l1_x;
    jn.Y = j.l1_y;
    if (nb > 0)
        hipLaunchKernelGGL(l1_normalize_kernel, dim3((unsigned)((nb + per - 1) / per)), dim3(256),
                           0, s, j, j.X, nb, j.l1_x);
    if (na > 0)
        hipLaunchKernelGGL(l1_normalize_kernel, dim3((unsigned)((na + per - 1) / per)), dim3(256),
                           0, s, j, j.Y, na, j.l1_y);
    const unsigned rows = (unsigned)((n_max + kTile - 1) / kTile);
    hipLaunchKernelGGL((points_tile_kernel<1, true>),
                       dim3((unsigned)((ldk_max + kTile - 1) / kTile), rows, 1), dim3(256), 0, s,
                       jn);
}

void launch_points_tiled(const PointsJob &j, int64_t n_max, int64_t ldk_max, hipStream_t s)
{
    const unsigned rows = (unsigned)((n_max + kTile - 1) / kTile);
    hipLaunchKernelGGL(points_tile_kernel<0>, dim3(rows, rows, j.batch), dim3(256), 0, s, j);
    hipLaunchKernelGGL(thresholds_kernel, dim3(threshold_blocks(j.kcap), 1, j.batch), dim3(256),
                       0, s, j);
    hipLaunchKernelGGL(points_tile_kernel<1>,
                       dim3((unsigned)((ldk_max + kTile - 1) / kTile), rows, j.batch), dim3(256),
                       0, s, j);
}

template <int D>
void launch_points_d(const PointsJob &j, int64_t n_max, int64_t ldk_max, hipStream_t s)
{
    PointsJob j_th = j;  // the thresholds pass: how many per-block maxima to reduce
    if (j.prune.cx && j.batch == 1) {
        const unsigned g = (unsigned)std::min<int64_t>(1024, (n_max + 255) / 256);
        hipLaunchKernelGGL(prune_reset_kernel, dim3(1), dim3(64), 0, s, j.prune);
        // few blocks: the extremes end in one set of atomics per block
        hipLaunchKernelGGL(extent_kernel<D>, dim3(std::min(g, 64u)), dim3(256), 0, s, j);
        hipLaunchKernelGGL(prune_kernel<D>, dim3(g), dim3(256), 0, s, j);
        PointsJob jm = j;
        jm.nmpart = kPairsMaxBlocks;
        hipLaunchKernelGGL(pairs_max_kernel<D>, dim3(kPairsMaxBlocks), dim3(kBuildThreads), 0, s,
                           jm);
        j_th.nmpart = kPairsMaxBlocks;
    } else {
        const int64_t per_block = (int64_t)kBuildThreads * kMaxCols;
        dim3 gmax((unsigned)((n_max + per_block - 1) / per_block),
                  (unsigned)((n_max + kMaxRows - 1) / kMaxRows), (unsigned)j.batch);
        if (j.mpart) {
            // row tiles strided so that at most max(kMaxParts, grid.x) maxima are stored
            gmax.y = std::max(1u, std::min(gmax.y, (unsigned)kMaxParts / gmax.x));
            j_th.nmpart = (int32_t)(gmax.x * gmax.y);
            j_th.nmpart_err = 1;
        }
        hipLaunchKernelGGL(points_max_kernel<D>, gmax, dim3(kBuildThreads), 0, s, j);
    }
    hipLaunchKernelGGL(thresholds_kernel, dim3(threshold_blocks(j.kcap), 1, j.batch), dim3(256),
                       0, s, j_th);
    if (j.no_matrix) return;
    const int64_t per_block = (int64_t)kBuildThreads * kColsPerThread;
    dim3 gk((unsigned)((ldk_max + per_block - 1) / per_block),
            (unsigned)((n_max + kRowsPerBlock - 1) / kRowsPerBlock), (unsigned)j.batch);
    hipLaunchKernelGGL(points_k_kernel<D>, gk, dim3(kBuildThreads), 0, s, j);
}

}  // namespace

hipError_t launch_round_costs(const float *C, int64_t n, int64_t na, int64_t ldc, double eps,
                              int16_t *k, int64_t ldk, Ctl *ctl, hipStream_t s, int k8)
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
        hipLaunchKernelGGL(round_costs_kernel, grid, dim3(kBuildThreads), 0, s, C, n, na, ldc,
                           eps, k, ldk, ctl, k8);
    return hipGetLastError();
}

hipError_t launch_points(const PointsJob &j, int64_t n_max, int64_t ldk_max, hipStream_t s)
{
    // The plain maximum pass of one instance (d = 2, 3) with per-block maxima
    // needs no reset: the thresholds pass writes m, K and the error word.
    const bool self_reset = j.mpart && !j.prune.cx && j.batch == 1 && n_max > 0 &&
                            (j.d == 2 || j.d == 3) && j.metric != 2;
    if (!self_reset)
        hipLaunchKernelGGL(build_reset_kernel, dim3((j.batch + 255) / 256), dim3(256), 0, s, j);
    if (n_max == 0 || j.batch == 0) return hipGetLastError();
    if (j.metric == 2) launch_points_l1(j, n_max, ldk_max, s);
    else if (j.d == 2) launch_points_d<2>(j, n_max, ldk_max, s);
    else if (j.d == 3) launch_points_d<3>(j, n_max, ldk_max, s);
    else if (j.mfma.tile_max) return launch_points_mfma(j, j.mfma, n_max, ldk_max, s);
    else launch_points_tiled(j, n_max, ldk_max, s);
    return hipGetLastError();
}

}  // namespace prot
