// Cosine similarity of first left singular vectors, the measure of the
// paper's case study of finding similar time ranges (Sec. 5): for a base
// range and earlier windows of the same length, u_1 of each window against
// u_1 of the base, row by row within the window.
#include "zs_internal.h"

namespace zs {
namespace {

// Deterministic sums of three values per thread over the work-group.
__device__ void block_sum3(double &a, double &b, double &c, double *red)
{
    const int tid = threadIdx.x;
    red[tid] = a;
    red[kThreads + tid] = b;
    red[2 * kThreads + tid] = c;
    __syncthreads();
    for (int s = kThreads / 2; s >= 1; s /= 2) {
        if (tid < s) {
            red[tid] += red[tid + s];
            red[kThreads + tid] += red[kThreads + tid + s];
            red[2 * kThreads + tid] += red[2 * kThreads + tid + s];
        }
        __syncthreads();
    }
    a = red[0];
    b = red[kThreads];
    c = red[2 * kThreads];
}

// U holds nw + 1 vectors of n elements back to back: u_1 of the base, then of
// windows 1..nw.  sim[w - 1] = <u_base, u_w> / (|u_base| |u_w|), or 0 when
// either vector is zero (a window of rank 0).  One work-group per window.
template <typename TU>
__global__ __launch_bounds__(kThreads) void cosine_kernel(const TU *__restrict__ U, int64_t n,
                                                          double *__restrict__ sim)
{
    __shared__ double red[3 * kThreads];
    const int w = blockIdx.x + 1;
    const TU *u0 = U;
    const TU *uw = U + (int64_t)w * n;
    double dot = 0.0, n0 = 0.0, nw = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kThreads) {
        const double x = (double)u0[i], y = (double)uw[i];
        dot = fma(x, y, dot);
        n0 = fma(x, x, n0);
        nw = fma(y, y, nw);
    }
    block_sum3(dot, n0, nw, red);
    if (threadIdx.x == 0) sim[blockIdx.x] = (n0 > 0.0 && nw > 0.0) ? dot / (sqrt(n0) * sqrt(nw)) : 0.0;
}

}  // namespace

hipError_t launch_cosine(const void *U, int u_f32, int64_t n, int nw, double *sim,
                         hipStream_t stream)
{
    if (nw <= 0) return hipSuccess;
    timing_begin("cosine", stream);
    if (u_f32)
        cosine_kernel<float><<<nw, kThreads, 0, stream>>>(static_cast<const float *>(U), n, sim);
    else
        cosine_kernel<double><<<nw, kThreads, 0, stream>>>(static_cast<const double *>(U), n, sim);
    hipError_t e = hipGetLastError();
    timing_end("cosine", stream);
    return e;
}

}  // namespace zs
