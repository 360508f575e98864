// Squared Euclidean costs on the matrix cores (d >= 16), bit-identical to
// the binary32 direct-difference definition used everywhere else
// (s = fma(x_j - y_j, x_j - y_j, s) in coordinate order, k = floor((s/m)/eps)
// with binary64 divisions; arXiv:2203.03732 Section 2.1, eq. (1)).
//
// MFMA computes a = |x|^2 + |y|^2 - 2<x, y> for a 64 x 64 tile of pairs
// (four waves, one 32 x 32 block each, v_mfma_f32_32x32x2_f32). Standard
// floating-point error bounds give |a - s| <= (2d + 6) u (|x| + |y|)^2 with
// u = 2^-24 for any summation order of the dot product; the code uses four
// times that, E = c (|x| + |y|)^2. Then:
//  * exact maximum: M~ = max a, E_max = max E; every tile whose largest a
//    reaches M~ - 2 E_max is recomputed with the definition, and the largest
//    exact value among them is m (the pair attaining m has a >= m - E_max
//    >= M~ - 2 E_max, since M~ <= m + E_max);
//  * rounded cost: with v = a * (1 / (m eps)), when v is farther than
//    E / (m eps) plus the binary32 classification margin from every integer,
//    floor(v) is the definition's k; otherwise the pair is recomputed with the
//    definition and classified against the exact threshold table.
#include "cost_common.h"
#include "internal.h"

#include <float.h>
#include <math.h>

namespace prot {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kT = 64;      // tile rows and columns
constexpr int kKC = 64;     // coordinates staged per step
constexpr int kPad = kKC + 1;

// Row i (0..31) of the 32 x 32 block held in accumulator v of lane l:
// column l % 32, row 8 (v / 4) + 4 (l / 32) + v % 4.
__device__ inline int acc_row(int v, int lane) { return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3); }

struct TileDots {
    floatx16 acc;
    int rbase, cbase;  // this wave's block inside the tile
};

// Stage the tile's coordinates chunk by chunk and accumulate the dot
// products of this wave's 32 x 32 block; also the squared norms of the
// tile's 64 rows and 64 columns (any order: they only enter the
// approximation).
__device__ inline TileDots tile_dots(const Instance &in, int d, int64_t b0, int64_t a0,
                                     float (*xs)[kPad], float (*ys)[kPad], float *nx, float *ny)
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    TileDots t;
    t.rbase = 32 * (w >> 1);
    t.cbase = 32 * (w & 1);
    for (int i = 0; i < 16; ++i) t.acc[i] = 0.0f;
    if (tid < kT) nx[tid] = 0.0f;
    else if (tid < 2 * kT) ny[tid - kT] = 0.0f;
    for (int k0 = 0; k0 < d; k0 += kKC) {
        __syncthreads();
        for (int q = tid; q < kT * kKC; q += 256) {
            const int r = q / kKC, c = q - r * kKC;
            const bool ok = k0 + c < d;
            xs[r][c] = (ok && b0 + r < in.n) ? in.X[(b0 + r) * d + k0 + c] : 0.0f;
            ys[r][c] = (ok && a0 + r < in.n) ? in.Y[(a0 + r) * d + k0 + c] : 0.0f;
        }
        __syncthreads();
        if (tid < kT) {
            float s = nx[tid];
            for (int c = 0; c < kKC; ++c) s = __fmaf_rn(xs[tid][c], xs[tid][c], s);
            nx[tid] = s;
        } else if (tid < 2 * kT) {
            const int r = tid - kT;
            float s = ny[r];
            for (int c = 0; c < kKC; ++c) s = __fmaf_rn(ys[r][c], ys[r][c], s);
            ny[r] = s;
        }
        const int row = lane & 31, kk = lane >> 5;
#pragma unroll 8
        for (int c = 0; c < kKC; c += 2) {
            const float a = xs[t.rbase + row][c + kk];
            const float b = ys[t.cbase + row][c + kk];
            t.acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, t.acc, 0, 0, 0);
        }
    }
    __syncthreads();
    return t;
}

__device__ inline float approx_at(const TileDots &t, int v, int lane, const float *nx,
                                  const float *ny, int &r, int &c)
{
    r = t.rbase + acc_row(v, lane);
    c = t.cbase + (lane & 31);
    return __fsub_rn(__fadd_rn(nx[r], ny[c]), __fmul_rn(2.0f, t.acc[v]));
}

__device__ inline float err_bound(float cE, float nxr, float nyc)
{
    const float s = __fadd_rn(__fsqrt_rn(nxr), __fsqrt_rn(nyc));
    return cE * s * s * 1.0001f;
}

// Pass A: approximate maximum and error bound of every instance; the largest
// approximate value of each tile.
__global__ void __launch_bounds__(256) mfma_max_kernel(PointsJob j, MfmaAux x)
{
    __shared__ float xs[kT][kPad], ys[kT][kPad];
    __shared__ float nx[kT], ny[kT];
    __shared__ float red_m[4], red_e[4];
    const Instance in = j.instance(blockIdx.z);
    const int64_t b0 = (int64_t)blockIdx.y * kT, a0 = (int64_t)blockIdx.x * kT;
    if (b0 >= in.n || a0 >= in.n) return;
    const TileDots t = tile_dots(in, j.d, b0, a0, xs, ys, nx, ny);
    const int lane = threadIdx.x & 63;
    float mx = 0.0f, ex = 0.0f;
    bool bad = false;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        int r, c;
        const float a = approx_at(t, v, lane, nx, ny, r, c);
        if (b0 + r < in.n && a0 + c < in.n) {
            bad |= !(a <= FLT_MAX && a >= -FLT_MAX);
            mx = fmaxf(mx, a);
            ex = fmaxf(ex, err_bound(x.cE, nx[r], ny[c]));
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        mx = fmaxf(mx, __shfl_xor(mx, off));
        ex = fmaxf(ex, __shfl_xor(ex, off));
    }
    if (lane == 0) {
        red_m[threadIdx.x >> 6] = mx;
        red_e[threadIdx.x >> 6] = ex;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const float m = fmaxf(fmaxf(red_m[0], red_m[1]), fmaxf(red_m[2], red_m[3]));
        const float e = fmaxf(fmaxf(red_e[0], red_e[1]), fmaxf(red_e[2], red_e[3]));
        x.tile_max[(int64_t)blockIdx.z * x.tiles_per_inst + (int64_t)blockIdx.y * x.tiles_x +
                   blockIdx.x] = m;
        __hip_atomic_fetch_max(reinterpret_cast<unsigned *>(&x.amax[blockIdx.z]),
                               __float_as_uint(m), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_max(reinterpret_cast<unsigned *>(&x.emax[blockIdx.z]),
                               __float_as_uint(e), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (bad) __hip_atomic_fetch_or(j.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Pass B: the definition on the tiles that can hold the maximum.
__global__ void __launch_bounds__(256) mfma_exact_max_kernel(PointsJob j, MfmaAux x)
{
    __shared__ float red[4];
    const Instance in = j.instance(blockIdx.z);
    const int64_t b0 = (int64_t)blockIdx.y * kT, a0 = (int64_t)blockIdx.x * kT;
    if (b0 >= in.n || a0 >= in.n) return;
    const float tm = x.tile_max[(int64_t)blockIdx.z * x.tiles_per_inst +
                                (int64_t)blockIdx.y * x.tiles_x + blockIdx.x];
    const float lim = x.amax[blockIdx.z] - 2.0f * x.emax[blockIdx.z];
    if (!(tm >= lim)) return;
    float mx = 0.0f;
    for (int q = threadIdx.x; q < kT * kT; q += 256) {
        const int r = q / kT, c = q - r * kT;
        if (b0 + r < in.n && a0 + c < in.n)
            mx = fmaxf(mx, sqdist<0>(in.X + (b0 + r) * j.d, in.Y + (a0 + c) * j.d, j.d));
    }
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
        __hip_atomic_fetch_max(reinterpret_cast<unsigned *>(&j.m[blockIdx.z]), __float_as_uint(m),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Pass C: rounded costs; uncertain pairs are recomputed with the definition.
__global__ void __launch_bounds__(256) mfma_k_kernel(PointsJob j, MfmaAux x)
{
    __shared__ float xs[kT][kPad], ys[kT][kPad];
    __shared__ float nx[kT], ny[kT];
    __shared__ __align__(16) int16_t ks[kT][kT + 8];
    const Instance in = j.instance(blockIdx.z);
    const int64_t b0 = (int64_t)blockIdx.y * kT, a0 = (int64_t)blockIdx.x * kT;
    if (b0 >= in.n || a0 >= in.ldk) return;
    const TileDots t = tile_dots(in, j.d, b0, a0, xs, ys, nx, ny);
    const int lane = threadIdx.x & 63;
    const float mf = j.m[blockIdx.z];
    const int32_t K = (mf > 0.0f) ? (int32_t)floor(1.0 / j.eps) : 0;
    const float inv = (mf > 0.0f) ? (float)(1.0 / ((double)mf * j.eps)) : 0.0f;
    const float base_margin = classify_margin(K) + 1e-6f;
    const float *th = j.th + (int64_t)blockIdx.z * j.kcap;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        int r, c;
        const float a = approx_at(t, v, lane, nx, ny, r, c);
        int g = 0x7FFF;
        if (b0 + r < in.n && a0 + c < in.n) {
            bool ok;
            g = fast_k(fmaxf(a, 0.0f), inv, base_margin + err_bound(x.cE, nx[r], ny[c]) * inv, K,
                       ok);
            ok = ok && a >= 0.0f;
            if (!ok) {
                const float s = sqdist<0>(in.X + (b0 + r) * j.d, in.Y + (a0 + c) * j.d, j.d);
                bool ok2;
                g = fast_k(s, inv, classify_margin(K), K, ok2);
                if (!ok2) g = refine_k(s, g, K, th);
            }
        }
        ks[r][c] = (int16_t)g;
    }
    __syncthreads();
    // 16-byte row segments: 8 per row, 512 per tile
    for (int q = threadIdx.x; q < kT * (kT / 8); q += 256) {
        const int r = q >> 3, c8 = (q & 7) * 8;
        if (b0 + r < in.n)
            *reinterpret_cast<uint4 *>(in.k + (b0 + r) * in.ldk + a0 + c8) =
                *reinterpret_cast<const uint4 *>(&ks[r][c8]);
    }
}

__global__ void mfma_reset_kernel(MfmaAux x, int32_t batch)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < batch; i += gridDim.x * blockDim.x) {
        x.amax[i] = 0.0f;
        x.emax[i] = 0.0f;
    }
}

__global__ void mfma_thresholds_kernel(PointsJob j)
{
    const float mf = j.m[blockIdx.z];
    const int32_t K = (mf > 0.0f) ? (int32_t)floor(1.0 / j.eps) : 0;
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && j.kmax_out && blockIdx.z == 0) *j.kmax_out = K;
    if (i > K + 1 || i >= j.kcap) return;
    j.th[(int64_t)blockIdx.z * j.kcap + i] = threshold_of(i, K, mf, j.eps);
}

}  // namespace

float mfma_error_constant(int32_t d) { return 4.0f * (2.0f * (float)d + 6.0f) * 5.9604645e-8f; }

hipError_t launch_points_mfma(const PointsJob &j, const MfmaAux &x, int64_t n_max,
                              int64_t ldk_max, hipStream_t s)
{
    hipLaunchKernelGGL(mfma_reset_kernel, dim3((j.batch + 255) / 256), dim3(256), 0, s, x, j.batch);
    const unsigned tiles = (unsigned)((n_max + kT - 1) / kT);
    hipLaunchKernelGGL(mfma_max_kernel, dim3(tiles, tiles, j.batch), dim3(256), 0, s, j, x);
    hipLaunchKernelGGL(mfma_exact_max_kernel, dim3(tiles, tiles, j.batch), dim3(256), 0, s, j, x);
    hipLaunchKernelGGL(mfma_thresholds_kernel, dim3((j.kcap + 255) / 256, 1, j.batch), dim3(256),
                       0, s, j);
    hipLaunchKernelGGL(mfma_k_kernel, dim3((unsigned)((ldk_max + kT - 1) / kT), tiles, j.batch),
                       dim3(256), 0, s, j, x);
    return hipGetLastError();
}

}  // namespace prot
