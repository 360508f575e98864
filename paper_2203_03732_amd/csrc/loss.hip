// Matching-based OT loss of a batch and its gradient.
//
// For instance i with matching mate_b (row b -> column a), the loss is
//   L_i = (1/n_i) * sum_b ||x_b - y_mate(b)||^2,
// the cost of the plan P = (1/n_i) * permutation that the push-relabel solve
// returns (arXiv:2203.03732 motivates using the plan in learning, Section 1).
// The plan is piecewise constant in X and Y, so for an upstream gradient g_i
//   dL/dx_b = (2 g_i / n_i) (x_b - y_mate(b)),
//   dL/dy_a = (2 g_i / n_i) (y_a - x_mate^-1(a)),
// and 0 for vertices the plan leaves unmatched.
#include "internal.h"

namespace prot {
namespace {

constexpr int kLossThreads = 256;
constexpr int kFwdThreads = 1024;
constexpr int kFwdUnroll = 4;

// One block per instance; coordinate e of the instance is handled by thread
// e mod kFwdThreads, so consecutive lanes read consecutive floats, with
// kFwdUnroll coordinates' loads in flight per thread. Binary64 accumulation
// (each thread in ascending e), fixed-order block reduction.
__global__ void __launch_bounds__(kFwdThreads)
ot_loss_fwd_kernel(LossArgs A, float *loss)
{
    __shared__ double red[kFwdThreads];
    const int inst = blockIdx.x;
    const int64_t n = A.n_arr[inst], off = A.pt_off[inst];
    const int d = A.d;
    const float *X = A.X + off * d, *Y = A.Y + off * d;
    const int32_t *mb = A.mate_b + off;
    const int64_t total = n * d;
    double s = 0.0;
    for (int64_t e0 = threadIdx.x; e0 < total; e0 += (int64_t)kFwdUnroll * kFwdThreads) {
        float x[kFwdUnroll], y[kFwdUnroll];
        bool use[kFwdUnroll];
#pragma unroll
        for (int u = 0; u < kFwdUnroll; ++u) {
            const int64_t e = e0 + (int64_t)u * kFwdThreads;
            use[u] = false;
            x[u] = y[u] = 0.0f;
            if (e < total) {
                const int64_t b = e / d;
                const int32_t a = mb[b];
                if (a >= 0) {
                    use[u] = true;
                    x[u] = X[e];
                    y[u] = Y[(int64_t)a * d + (e - b * d)];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kFwdUnroll; ++u)
            if (use[u]) {
                const double t = __dsub_rn((double)x[u], (double)y[u]);
                s = __dadd_rn(s, __dmul_rn(t, t));
            }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = kFwdThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] = __dadd_rn(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[inst] = n > 0 ? (float)(red[0] / (double)n) : 0.0f;
}

// grid.y = instance, grid.x over the instance's n * d coordinates.
__global__ void __launch_bounds__(kLossThreads)
ot_loss_bwd_kernel(LossArgs A, const float *grad_loss, float *dX, float *dY)
{
    const int inst = blockIdx.y;
    const int64_t n = A.n_arr[inst], off = A.pt_off[inst];
    const int d = A.d;
    const int64_t e = (int64_t)blockIdx.x * kLossThreads + threadIdx.x;
    if (e >= n * d) return;
    const int64_t v = e / d;
    const int j = (int)(e - v * d);
    const float scale = 2.0f * grad_loss[inst] / (float)n;
    const float *X = A.X + off * d, *Y = A.Y + off * d;
    const int32_t a = A.mate_b[off + v];
    const int32_t b = A.mate_a[off + v];
    dX[off * d + e] = a >= 0 ? scale * (X[e] - Y[(int64_t)a * d + j]) : 0.0f;
    dY[off * d + e] = b >= 0 ? scale * (Y[e] - X[(int64_t)b * d + j]) : 0.0f;
}

}  // namespace

hipError_t launch_loss_fwd(const LossArgs &a, float *loss, hipStream_t s)
{
    if (a.batch > 0)
        hipLaunchKernelGGL(ot_loss_fwd_kernel, dim3(a.batch), dim3(kFwdThreads), 0, s, a, loss);
    return hipGetLastError();
}

hipError_t launch_loss_bwd(const LossArgs &a, int64_t n_max, const float *grad_loss, float *dX,
                           float *dY, hipStream_t s)
{
    if (a.batch > 0) {
        const int64_t blocks = (n_max * a.d + kLossThreads - 1) / kLossThreads;
        hipLaunchKernelGGL(ot_loss_bwd_kernel, dim3((unsigned)blocks, (unsigned)a.batch),
                           dim3(kLossThreads), 0, s, a, grad_loss, dX, dY);
    }
    return hipGetLastError();
}

}  // namespace prot
