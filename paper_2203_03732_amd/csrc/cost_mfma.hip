// Squared Euclidean costs on the matrix cores (d >= 16), bit-identical to
// the binary32 direct-difference definition used everywhere else
// (s = fma(x_j - y_j, x_j - y_j, s) in coordinate order, k = floor((s/m)/eps)
// with binary64 divisions; arXiv:2203.03732 Section 2.1, eq. (1)).
//
// The matrix cores compute a = |x|^2 + |y|^2 - 2<x, y> for a 128 x 128 tile
// of pairs per workgroup: four waves, each a 64 x 64 quarter made of 2 x 2
// blocks of v_mfma_f32_32x32x2_f32, so that every operand read from LDS
// feeds two matrix instructions. The tile's coordinates are staged through
// LDS 64 at a time, transposed (coordinate-major), so that the 32 lanes
// reading one operand column touch 32 consecutive words; for d <= 64 the
// whole tile stays in LDS, where the exact recomputations read it. The squared norms
// of the tile's rows and columns are summed from the same staged values.
// Standard floating-point error bounds give |a - s| <= (2d + 6) u (|x| +
// |y|)^2 with u = 2^-24 for any summation order of the dot product; the
// code uses four times that, E = c (|x| + |y|)^2. Then:
//  * exact maximum: M~ = max a, E_max = max E; in every tile whose largest a
//    reaches M~ - 2 E_max, the pairs whose a reaches it are recomputed with
//    the definition, and the largest exact value among them is m (the pair
//    attaining m has a >= m - E_max >= M~ - 2 E_max, since M~ <= m + E_max);
//  * rounded cost: with v = a * (1 / (m eps)), when v is farther than
//    E / (m eps) plus the binary32 classification margin from every integer,
//    floor(v) is the definition's k; otherwise the pair is marked, and after
//    the tile is classified the workgroup recomputes the marked pairs with the
//    definition and classifies them against the exact threshold table.
#include "cost_common.h"
#include "internal.h"

#include <float.h>
#include <math.h>

namespace prot {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kT = (int)kMfmaTile;  // tile rows and columns (128)
constexpr int kKC = 64;              // coordinates staged per step (d <= 64: all of them)
constexpr int kList = 2048;          // uncertain entries of a tile settled together
constexpr int kLd = kT + 4;          // floats per staged coordinate (row of the transposed stage)
constexpr int kKs = kT + 8;          // int16 per row of the output tile

static_assert(kT == 128, "four waves of 2 x 2 blocks of 32 x 32");

// LDS of a tile: the transposed stages while the dot products accumulate,
// then (pass C) the rounded tile on its way out; the norms and their roots
// (for the error bound) throughout.
struct StageLds {
    float xs[kKC][kLd];  // xs[k][r] = X[b0 + r][k0 + k]
    float ys[kKC][kLd];  // ys[k][c] = Y[a0 + c][k0 + k]
};
constexpr size_t kTileLds = sizeof(StageLds) > sizeof(int16_t) * kT * kKs
                                ? sizeof(StageLds)
                                : sizeof(int16_t) * kT * kKs;

// Row i (0..31) of the 32 x 32 block held in accumulator v of lane l:
// column l % 32, row 8 (v / 4) + 4 (l / 32) + v % 4.
__device__ inline int acc_row(int v, int lane) { return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3); }

// The dot products of this wave's 64 x 64 quarter of the tile (blocks
// acc[2 i + j], rows 64 wr + 32 i, columns 64 wc + 32 j) and the squared
// norms and their roots of the tile's 128 rows (nx, sx) and columns (ny, sy).
__device__ inline void tile_dots(const Instance &in, int d, int64_t b0, int64_t a0, StageLds &st,
                                 float *nx, float *ny, float *sx, float *sy, floatx16 (&acc)[4])
{
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = w >> 1, wc = w & 1;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[q][i] = 0.0f;
    float norm = 0.0f;  // thread t < 128: row t; else column t - 128
    const int row = lane & 31, kk = lane >> 5;
    for (int k0 = 0; k0 < d; k0 += kKC) {
        // coordinates of this step, rounded up to a multiple of 8 (four
        // matrix steps; the staged values past d are 0)
        const int kc = min(kKC, (d - k0 + 7) & ~7);
        __syncthreads();
        // 128 points x kc coordinates per side: runs of consecutive
        // coordinates of one point (coalesced reads, 16 bytes at a time when
        // d is a multiple of 4), stored transposed
        if ((d & 3) == 0) {
            const int kc4 = kc >> 2;
            for (int q = tid; q < kT * kc4; q += 256) {
                const int r = q / kc4, c = (q - r * kc4) * 4;
                const bool ok = k0 + c < d;  // d % 4 == 0: all four or none
                float4 xv = make_float4(0.0f, 0.0f, 0.0f, 0.0f), yv = xv;
                if (ok && b0 + r < in.n)
                    xv = *reinterpret_cast<const float4 *>(in.X + (b0 + r) * d + k0 + c);
                if (ok && a0 + r < in.na)
                    yv = *reinterpret_cast<const float4 *>(in.Y + (a0 + r) * d + k0 + c);
                st.xs[c][r] = xv.x;
                st.xs[c + 1][r] = xv.y;
                st.xs[c + 2][r] = xv.z;
                st.xs[c + 3][r] = xv.w;
                st.ys[c][r] = yv.x;
                st.ys[c + 1][r] = yv.y;
                st.ys[c + 2][r] = yv.z;
                st.ys[c + 3][r] = yv.w;
            }
        } else {
            for (int q = tid; q < kT * kc; q += 256) {
                const int r = q / kc, c = q - r * kc;
                const bool ok = k0 + c < d;
                st.xs[c][r] = (ok && b0 + r < in.n) ? in.X[(b0 + r) * d + k0 + c] : 0.0f;
                st.ys[c][r] = (ok && a0 + r < in.na) ? in.Y[(a0 + r) * d + k0 + c] : 0.0f;
            }
        }
        __syncthreads();
        {
            const float(*src)[kLd] = tid < kT ? st.xs : st.ys;
            const int p = tid & (kT - 1);
#pragma unroll 8
            for (int c = 0; c < kc; ++c) norm = __fmaf_rn(src[c][p], src[c][p], norm);
        }
        for (int c8 = 0; c8 < kc; c8 += 8) {
#pragma unroll
            for (int c = c8; c < c8 + 8; c += 2) {
                const float a0v = st.xs[c + kk][64 * wr + row];
                const float a1v = st.xs[c + kk][64 * wr + 32 + row];
                const float b0v = st.ys[c + kk][64 * wc + row];
                const float b1v = st.ys[c + kk][64 * wc + 32 + row];
                acc[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0v, b0v, acc[0], 0, 0, 0);
                acc[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0v, b1v, acc[1], 0, 0, 0);
                acc[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1v, b0v, acc[2], 0, 0, 0);
                acc[3] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1v, b1v, acc[3], 0, 0, 0);
            }
        }
    }
    if (tid < kT) {
        nx[tid] = norm;
        sx[tid] = __fsqrt_rn(norm);
    } else {
        ny[tid - kT] = norm;
        sy[tid - kT] = __fsqrt_rn(norm);
    }
    __syncthreads();
}

// Tile position of accumulator v of block q of this lane's wave.
__device__ inline void acc_pos(int q, int v, int lane, int w, int &r, int &c)
{
    r = 64 * (w >> 1) + 32 * (q >> 1) + acc_row(v, lane);
    c = 64 * (w & 1) + 32 * (q & 1) + (lane & 31);
}

// The definition for one pair: fma-accumulated squared differences in
// coordinate order (a sequential chain; the loads are independent and go out
// ahead of it).
__device__ inline float exact_d2(const float *__restrict__ x, const float *__restrict__ y, int d)
{
    float s = 0.0f;
    int j = 0;
    for (; j + 8 <= d; j += 8) {
        float t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = __fsub_rn(x[j + u], y[j + u]);
#pragma unroll
        for (int u = 0; u < 8; ++u) s = __fmaf_rn(t[u], t[u], s);
    }
    for (; j < d; ++j) {
        const float t = __fsub_rn(x[j], y[j]);
        s = __fmaf_rn(t, t, s);
    }
    return s;
}

__device__ inline float err_bound(float cE, float sxr, float syc)
{
    const float s = __fadd_rn(sxr, syc);
    return cE * s * s * 1.0001f;
}

// Pass A: approximate maximum and error bound of every instance; the largest
// approximate value of each tile.
__global__ void __launch_bounds__(256) mfma_max_kernel(PointsJob j, MfmaAux x)
{
    __shared__ __align__(16) char lds[kTileLds];
    __shared__ float nx[kT], ny[kT], sx[kT], sy[kT];
    __shared__ float red_m[4], red_e[4];
    const Instance in = j.instance(blockIdx.z);
    const int64_t b0 = (int64_t)blockIdx.y * kT, a0 = (int64_t)blockIdx.x * kT;
    if (b0 >= in.n || a0 >= in.na) return;
    floatx16 acc[4];
    tile_dots(in, j.d, b0, a0, *reinterpret_cast<StageLds *>(lds), nx, ny, sx, sy, acc);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    float mx = 0.0f, ex = 0.0f;
    bool bad = false;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            int r, c;
            acc_pos(q, v, lane, w, r, c);
            if (b0 + r < in.n && a0 + c < in.na) {
                const float a = __fsub_rn(__fadd_rn(nx[r], ny[c]), __fmul_rn(2.0f, acc[q][v]));
                bad |= !(a <= FLT_MAX && a >= -FLT_MAX);
                mx = fmaxf(mx, a);
            }
        }
    // the error bound of every pair of the tile is at most the bound taken
    // with the tile's largest norms (E grows with |x| + |y|)
    {
        const int r = threadIdx.x & (kT - 1);
        if (threadIdx.x < kT ? b0 + r < in.n : a0 + r < in.na)
            ex = threadIdx.x < kT ? sx[r] : sy[r];
    }
    for (int off = 32; off > 0; off >>= 1) {
        mx = fmaxf(mx, __shfl_xor(mx, off));
        ex = fmaxf(ex, __shfl_xor(ex, off));
    }
    if (lane == 0) {
        red_m[w] = mx;
        red_e[w] = ex;  // waves 0, 1: largest root norm of a row; 2, 3: of a column
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const float m = fmaxf(fmaxf(red_m[0], red_m[1]), fmaxf(red_m[2], red_m[3]));
        const float e = err_bound(x.cE, fmaxf(red_e[0], red_e[1]), fmaxf(red_e[2], red_e[3]));
        x.tile_max[(int64_t)blockIdx.z * x.tiles_per_inst + (int64_t)blockIdx.y * x.tiles_x +
                   blockIdx.x] = m;
        __hip_atomic_fetch_max(reinterpret_cast<unsigned *>(&x.amax[blockIdx.z]),
                               __float_as_uint(m), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_max(reinterpret_cast<unsigned *>(&x.emax[blockIdx.z]),
                               __float_as_uint(e), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (bad) __hip_atomic_fetch_or(j.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Pass B: on the tiles that can hold the maximum, the approximation again,
// and the definition for the pairs whose approximation can be the maximum
// (a >= M~ - 2 E_max).
__global__ void __launch_bounds__(256) mfma_exact_max_kernel(PointsJob j, MfmaAux x)
{
    __shared__ __align__(16) char lds[kTileLds];
    __shared__ float nx[kT], ny[kT], sx[kT], sy[kT];
    __shared__ float red[4];
    const Instance in = j.instance(blockIdx.z);
    const int64_t b0 = (int64_t)blockIdx.y * kT, a0 = (int64_t)blockIdx.x * kT;
    if (b0 >= in.n || a0 >= in.na) return;
    const float tm = x.tile_max[(int64_t)blockIdx.z * x.tiles_per_inst +
                                (int64_t)blockIdx.y * x.tiles_x + blockIdx.x];
    const float lim = x.amax[blockIdx.z] - 2.0f * x.emax[blockIdx.z];
    if (!(tm >= lim)) return;
    floatx16 acc[4];
    tile_dots(in, j.d, b0, a0, *reinterpret_cast<StageLds *>(lds), nx, ny, sx, sy, acc);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    float mx = 0.0f;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            int r, c;
            acc_pos(q, v, lane, w, r, c);
            if (b0 + r < in.n && a0 + c < in.na) {
                const float a = __fsub_rn(__fadd_rn(nx[r], ny[c]), __fmul_rn(2.0f, acc[q][v]));
                if (a >= lim)
                    mx = fmaxf(mx, exact_d2(in.X + (b0 + r) * j.d, in.Y + (a0 + c) * j.d, j.d));
            }
        }
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    if (lane == 0) red[w] = mx;
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
    __shared__ __align__(16) char lds[kTileLds];
    __shared__ float nx[kT], ny[kT], sx[kT], sy[kT];
    const Instance in = j.instance(blockIdx.z);
    const int64_t b0 = (int64_t)blockIdx.y * kT, a0 = (int64_t)blockIdx.x * kT;
    if (b0 >= in.n || a0 >= in.ldk) return;
    floatx16 acc[4];
    tile_dots(in, j.d, b0, a0, *reinterpret_cast<StageLds *>(lds), nx, ny, sx, sy, acc);
    StageLds &st = *reinterpret_cast<StageLds *>(lds);
    __shared__ uint16_t list[kList];     // tile positions r * kT + c to settle
    __shared__ int16_t settled[kList];   // their rounded costs
    __shared__ uint32_t s_cnt;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const float mf = j.m[blockIdx.z];
    const int32_t K = (mf > 0.0f) ? (int32_t)floor(1.0 / j.eps) : 0;
    const float inv = (mf > 0.0f) ? (float)(1.0 / ((double)mf * j.eps)) : 0.0f;
    const float base_margin = classify_margin(K) + 1e-6f;
    const float *th = j.th + (int64_t)blockIdx.z * j.kcap;
    // the whole tile is in LDS when one step staged every coordinate
    const bool resident = j.d <= kKC;
    // the rounded cost of pair (r, c) by the definition, its coordinates
    // from LDS (while the stage holds the whole tile) or from global memory
    auto settle = [&](int r, int c, bool lds_ok) -> int {
        float s = 0.0f;
        if (lds_ok) {
            for (int k = 0; k < j.d; ++k) {
                const float t = __fsub_rn(st.xs[k][r], st.ys[k][c]);
                s = __fmaf_rn(t, t, s);
            }
        } else {
            s = exact_d2(in.X + (b0 + r) * j.d, in.Y + (a0 + c) * j.d, j.d);
        }
        bool ok;
        const int g = fast_k(s, inv, classify_margin(K), K, ok);
        return ok ? g : refine_k(s, g, K, th);
    };
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    // An entry the approximation places keeps its rounded cost in its
    // accumulator (as integer bits); the others go to the list (-1) or,
    // beyond the list's length, are marked -2 and settled at the end.
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            int r, c;
            acc_pos(q, v, lane, w, r, c);
            int g = 0x7FFF;
            if (b0 + r < in.n && a0 + c < in.na) {
                const float a = __fsub_rn(__fadd_rn(nx[r], ny[c]), __fmul_rn(2.0f, acc[q][v]));
                bool ok;
                g = fast_k(fmaxf(a, 0.0f), inv,
                           base_margin + err_bound(x.cE, sx[r], sy[c]) * inv, K, ok);
                if (!(ok && a >= 0.0f)) {
                    const uint32_t i = atomicAdd(&s_cnt, 1u);
                    g = -2;
                    if (i < (uint32_t)kList) {
                        list[i] = (uint16_t)(r * kT + c);
                        g = -1;
                    }
                }
            }
            acc[q][v] = __int_as_float(g);
        }
    __syncthreads();
    // the listed entries with the definition, spread over the workgroup
    const uint32_t cnt = min(s_cnt, (uint32_t)kList);
    for (uint32_t i = threadIdx.x; i < cnt; i += 256) {
        const int pos = list[i];
        settled[i] = (int16_t)settle(pos / kT, pos % kT, resident);
    }
    // every read of the staged coordinates is done: the rounded tile takes
    // their place
    __syncthreads();
    int16_t(*ks)[kKs] = reinterpret_cast<int16_t(*)[kKs]>(lds);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            int r, c;
            acc_pos(q, v, lane, w, r, c);
            const int g = __float_as_int(acc[q][v]);
            if (g != -1) ks[r][c] = (int16_t)g;
        }
    for (uint32_t i = threadIdx.x; i < cnt; i += 256) {
        const int pos = list[i];
        ks[pos / kT][pos % kT] = settled[i];
    }
    __syncthreads();
    if (s_cnt > (uint32_t)kList) {
        // more uncertain entries than the list holds (far from typical
        // inputs): the rest from global memory
        for (int q = threadIdx.x; q < kT * kT; q += 256) {
            const int r = q / kT, c = q - r * kT;
            if (ks[r][c] == -2) ks[r][c] = (int16_t)settle(r, c, false);
        }
        __syncthreads();
    }
    // 16-byte row segments: 16 per row, 2048 per tile
    for (int q = threadIdx.x; q < kT * (kT / 8); q += 256) {
        const int r = q >> 4, c8 = (q & 15) * 8;
        if (b0 + r < in.n && a0 + c8 < in.ldk)
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
