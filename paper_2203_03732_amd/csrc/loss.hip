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
#include <algorithm>
#include <mutex>

#include "internal.h"

// Partial sums of prot_ot_loss_fwd_static: a fixed array of the library, one
// copy per device, so that the call allocates nothing. In host code its name
// is only a handle: kernels get the device address from static_loss_partials.
static __device__ __align__(256) double scratch[prot::kStaticLossParts];

namespace prot {
namespace {

constexpr int kLossThreads = 256;
constexpr int kFwdThreads = 256;
constexpr int kFwdUnroll = 4;

__device__ inline int64_t inst_n(const LossArgs &A, int inst)
{
    return A.n_arr ? (int64_t)A.n_arr[inst] : A.n_uniform;
}
__device__ inline int64_t inst_off(const LossArgs &A, int inst)
{
    return A.n_arr ? A.pt_off[inst] : (int64_t)inst * A.n_uniform;
}

// grid (parts, batch): block `part` of instance `inst` sums the squared
// differences of coordinates [part * per, (part + 1) * per) of the instance
// (row-major, so consecutive lanes read consecutive floats, kFwdUnroll
// loads in flight per thread), each thread in ascending order in binary64,
// then a fixed-order block reduction into partial[inst * parts + part].
__global__ void __launch_bounds__(kFwdThreads)
ot_loss_part_kernel(LossArgs A, double *partial)
{
    __shared__ double red[kFwdThreads];
    const int inst = blockIdx.y, parts = gridDim.x;
    const int64_t n = inst_n(A, inst), off = inst_off(A, inst);
    const int d = A.d;
    const float *X = A.X + off * d, *Y = A.Y + off * d;
    const int32_t *mb = A.mate_b + off;
    const int64_t total = n * d;
    const int64_t per = (total + parts - 1) / parts;
    const int64_t lo = min(total, (int64_t)blockIdx.x * per), hi = min(total, lo + per);
    double s = 0.0;
    for (int64_t e0 = lo + threadIdx.x; e0 < hi; e0 += (int64_t)kFwdUnroll * kFwdThreads) {
        float x[kFwdUnroll], y[kFwdUnroll];
        bool use[kFwdUnroll];
#pragma unroll
        for (int u = 0; u < kFwdUnroll; ++u) {
            const int64_t e = e0 + (int64_t)u * kFwdThreads;
            use[u] = false;
            x[u] = y[u] = 0.0f;
            if (e < hi) {
                const int64_t b = e / d;
                const int32_t a = mb[b];
                if (a >= 0 && a < n) {
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
    if (threadIdx.x == 0) partial[(int64_t)inst * parts + blockIdx.x] = red[0];
}

// One thread per instance: the partial sums in part order, divided by n.
__global__ void ot_loss_sum_kernel(LossArgs A, const double *partial, int parts, float *loss)
{
    const int inst = blockIdx.x * blockDim.x + threadIdx.x;
    if (inst >= A.batch) return;
    double s = 0.0;
    for (int q = 0; q < parts; ++q) s = __dadd_rn(s, partial[(int64_t)inst * parts + q]);
    const int64_t n = inst_n(A, inst);
    loss[inst] = n > 0 ? (float)(s / (double)n) : 0.0f;
}

// grid.y = instance, grid.x over the instance's n * d coordinates.
__global__ void __launch_bounds__(kLossThreads)
ot_loss_bwd_kernel(LossArgs A, const float *grad_loss, float *dX, float *dY)
{
    const int inst = blockIdx.y;
    const int64_t n = inst_n(A, inst), off = inst_off(A, inst);
    const int d = A.d;
    const int64_t e = (int64_t)blockIdx.x * kLossThreads + threadIdx.x;
    if (e >= n * d) return;
    const int64_t v = e / d;
    const int j = (int)(e - v * d);
    const float scale = 2.0f * grad_loss[inst] / (float)n;
    const float *X = A.X + off * d, *Y = A.Y + off * d;
    const int32_t a = A.mate_b[off + v];
    const int32_t b = A.mate_a[off + v];
    dX[off * d + e] = a >= 0 && a < n ? scale * (X[e] - Y[(int64_t)a * d + j]) : 0.0f;
    dY[off * d + e] = b >= 0 && b < n ? scale * (Y[e] - X[(int64_t)b * d + j]) : 0.0f;
}

// Without mate_a: every coordinate of dY starts at 0 (a column no row
// holds keeps it), then each matched row b writes dX_b and the coordinates
// of its column's dY (a matching gives each column at most one row).
__global__ void fill_zero_kernel(float *p, int64_t count)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

__global__ void __launch_bounds__(kLossThreads)
ot_loss_bwd_rows_kernel(LossArgs A, const float *grad_loss, float *dX, float *dY)
{
    const int inst = blockIdx.y;
    const int64_t n = inst_n(A, inst), off = inst_off(A, inst);
    const int d = A.d;
    const int64_t e = (int64_t)blockIdx.x * kLossThreads + threadIdx.x;
    if (e >= n * d) return;
    const int64_t v = e / d;
    const int j = (int)(e - v * d);
    const float scale = 2.0f * grad_loss[inst] / (float)n;
    const float *X = A.X + off * d, *Y = A.Y + off * d;
    const int32_t a = A.mate_b[off + v];
    if (a >= 0 && a < n) {
        const float diff = X[e] - Y[(int64_t)a * d + j];
        dX[off * d + e] = scale * diff;
        dY[(off + a) * d + j] = -(scale * diff);
    } else {
        dX[off * d + e] = 0.0f;
    }
}

}  // namespace

int loss_parts(int64_t n_max, int32_t d)
{
    // about 8192 coordinates per block, at most 64 blocks per instance
    const int64_t p = (n_max * d + 8191) / 8192;
    return (int)(p < 1 ? 1 : (p > 64 ? 64 : p));
}

hipError_t launch_loss_fwd(const LossArgs &a, int64_t n_max, double *partial, float *loss,
                           hipStream_t s)
{
    if (a.batch > 0) {
        const int parts = loss_parts(n_max, a.d);
        hipLaunchKernelGGL(ot_loss_part_kernel, dim3((unsigned)parts, (unsigned)a.batch),
                           dim3(kFwdThreads), 0, s, a, partial);
        hipLaunchKernelGGL(ot_loss_sum_kernel, dim3((unsigned)((a.batch + 255) / 256)), dim3(256),
                           0, s, a, (const double *)partial, parts, loss);
    }
    return hipGetLastError();
}

// Device address of this device's copy of `scratch` (the device current on
// the calling thread), looked up once per device.
hipError_t static_loss_partials(double **out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double *ptr[kMaxDevices] = {};
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        ptr[dev] = static_cast<double *>(p);
    }
    *out = ptr[dev];
    return hipSuccess;
}

hipError_t launch_loss_bwd(const LossArgs &a, int64_t n_max, const float *grad_loss, float *dX,
                           float *dY, hipStream_t s)
{
    if (a.batch > 0) {
        const int64_t blocks = (n_max * a.d + kLossThreads - 1) / kLossThreads;
        if (a.mate_a) {
            hipLaunchKernelGGL(ot_loss_bwd_kernel, dim3((unsigned)blocks, (unsigned)a.batch),
                               dim3(kLossThreads), 0, s, a, grad_loss, dX, dY);
        } else {
            const int64_t count = (int64_t)a.batch * n_max * a.d;  // uniform n
            const int64_t g = std::min<int64_t>((count + 255) / 256, 65536);
            hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)g), dim3(256), 0, s, dY, count);
            hipLaunchKernelGGL(ot_loss_bwd_rows_kernel, dim3((unsigned)blocks, (unsigned)a.batch),
                               dim3(kLossThreads), 0, s, a, grad_loss, dX, dY);
        }
    }
    return hipGetLastError();
}

}  // namespace prot
