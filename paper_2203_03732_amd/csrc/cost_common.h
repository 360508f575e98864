// Device helpers for the rounded-cost definitions of the point-set builds
// (arXiv:2203.03732, Section 2.1, eq. (1), on costs scaled to max 1).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace prot {

// One instance of a (possibly batched) point-set cost build.
struct Instance {
    const float *X;   // n x d rows (supply B)
    const float *Y;   // na x d columns (demand A)
    int64_t n;        // rows
    int64_t na;       // columns (na >= n; = n except for unbalanced single instances)
    int64_t ldk;      // row pitch of its rounded-cost matrix
    int16_t *k;
};

// Workspace of the matrix-core path (d >= 16), per instance.
struct MfmaAux {
    float *amax;              // largest approximate squared distance
    float *emax;              // largest error bound
    float *tile_max;          // per 64 x 64 tile: largest approximate value
    int64_t tiles_per_inst;   // tiles_x * tiles_x
    int32_t tiles_x;          // 64-wide tiles along n_max
    float cE;                 // error-bound constant for this d
};

// Workspace of the pruned maximum (one instance, d <= 3).
struct PruneAux {
    unsigned long long *ext;  // [16]: X then Y, per direction u: (order(u . p) << 32) | index
    uint32_t *bb;             // [12]: order-encoded min X, max X, min Y, max Y per coordinate
    uint32_t *cnt;            // [2]: candidate counts of X and Y
    int32_t *cx, *cy;         // candidate indices (n each)
};

struct PointsJob {
    const float *X, *Y;        // packed points; instance i starts at row pt_off[i]
    const int64_t *pt_off;     // device, per instance (null: one instance at row 0)
    const int32_t *n_arr;      // device, per instance (null: n_single)
    const int64_t *k_off;      // device, element offset of each instance's matrix
    const int32_t *ldk_arr;    // device, row pitch per instance (null: ldk_single)
    int64_t n_single, ldk_single;
    int64_t na_single;         // columns of a single instance (0: n_single)
    // Cost of a pair (Section 5's variants): 0 squared Euclidean d2 / m,
    // 1 Euclidean sqrt(d2 / m), 2 half the L1 distance of the vectors
    // normalised to sum 1 (X and Y then point at the normalised copies).
    int32_t metric;
    int32_t k8;                // 1: write k as uint8 (K <= 253, padding 0xFF); single instance
    float *l1_x, *l1_y;        // metric 2: workspace for the normalised X and Y
    int32_t d;
    int32_t batch;
    double eps;
    int16_t *k;
    float *m;                  // per instance: max squared distance
    float *th;                 // per instance: kcap thresholds
    int32_t kcap;              // floor(1 / eps) + 2
    int32_t *err;              // bit 0 set on a non-finite distance
    int32_t *kmax_out;         // optional: K of instance 0
    MfmaAux mfma;              // used when mfma.tile_max is set (d >= 16)
    int32_t no_matrix;         // 1: maximum and thresholds only (costs computed on the fly)
    PruneAux prune;            // used when prune.cx is set (one instance, d = 2, 3)
    float *mpart;              // one instance, d = 2, 3: per-block maxima (else atomics on m)
    int32_t nmpart;            // how many of them the thresholds pass reduces
    int32_t nmpart_err;        // 1: they carry the error flag (-1), the thresholds pass sets err

    __device__ Instance instance(int i) const
    {
        Instance in;
        const int64_t off = pt_off ? pt_off[i] : 0;
        in.X = X + off * d;
        in.Y = Y + off * d;
        in.n = n_arr ? n_arr[i] : n_single;
        in.na = (n_arr || na_single == 0) ? in.n : na_single;
        in.ldk = ldk_arr ? ldk_arr[i] : ldk_single;
        in.k = k + (k_off ? k_off[i] : 0);
        return in;
    }
};

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

// k(s) = floor((s / m) / eps), both divisions binary64 (the definition);
// Euclidean (metric 1): floor(sqrt(s / m) / eps), also binary64.
__device__ inline double k_of(float s, double m, double eps, int metric = 0)
{
    const double c = (double)s / m;
    return floor((metric == 1 ? sqrt(c) : c) / eps);
}

// Smallest binary32 s >= 0 with k(s) >= j (0 < j <= K); j = 0 gives 0 and
// j = K + 1 gives +inf. k(s) is non-decreasing in s, hence in the bit
// pattern of s >= 0, and k(m) = K.
__device__ inline float threshold_of(int32_t j, int32_t K, float mf, double eps, int metric = 0)
{
    if (j == 0) return 0.0f;
    if (j > K) return __int_as_float(0x7f800000);
    const double m = (double)mf;
    uint32_t lo = 0, hi = __float_as_uint(mf);
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (k_of(__uint_as_float(mid), m, eps, metric) >= (double)j) hi = mid;
        else lo = mid + 1;
    }
    return __uint_as_float(lo);
}

// v = s * inv in binary32 is within (K + 2) * 2^-22 of the exact s / (m eps)
// for every 0 <= s <= m (inv and the product are each rounded once; the exact
// value is <= K + 1), and the binary64 definition is within 1e-10 of it. So
// when v is at least this margin away from every integer, floor(v) is the
// definition's k (at most K, since s <= m).
__device__ inline float classify_margin(int32_t K) { return (float)(K + 2) * 4.8e-7f; }

__device__ inline int fast_k(float s, float inv, float delta, int K, bool &exact)
{
    const float v = __fmul_rn(s, inv);
    // v - floor(v), exact for 0 <= v < 2^23; floor(v) by truncation (v >= 0)
    const float f = __builtin_amdgcn_fractf(v);
    const int g = (int)v;
    exact = f >= delta && f <= 1.0f - delta;
    (void)K;
    return g;
}

// Exact k from a starting guess (clamped to [0, K]) and the threshold table
// th[0..K+1].
__device__ inline int refine_k(float s, int g, int K, const float *th)
{
    g = g > K ? K : (g < 0 ? 0 : g);
    while (g < K && s >= th[g + 1]) ++g;
    while (g > 0 && s < th[g]) --g;
    return g;
}

}  // namespace prot
