// Projection of the data on the first-stage eigenvectors, and the in-place
// U formation of the storage phase.
//
//  * project: for a chunk of rows of X (a block of A, or a query's stack M),
//    Y = X V_k (rows x kk, written out) and the partial Gram Y^T Y (kk x kk,
//    one slot per chunk).  X rows are staged through LDS with coalesced
//    loads; V_k sits in LDS for the whole chunk.
//  * utransform: U_(i) <- Y_(i) F_(i) in place (F = W Sigma^-1 with the sign
//    rule folded in), giving the block's left singular vectors.
#include "zs_internal.h"

namespace zs {
namespace {

constexpr int PR_RB = 16;   // rows staged per step

__global__ __launch_bounds__(kThreads) void project_kernel(const double *__restrict__ X, int64_t ld,
                                                           int c, const Chunk *__restrict__ chunks,
                                                           const double *__restrict__ Vk,
                                                           double *__restrict__ Y,
                                                           double *__restrict__ GYpart)
{
    extern __shared__ __align__(16) double smem[];
    const Chunk ch = chunks[blockIdx.x];
    const int kk = ch.kk;
    double *Vs = smem;                    // c x kk
    double *Xs = Vs + c * kk;             // PR_RB x c
    double *Ys = Xs + PR_RB * c;          // PR_RB x kk
    const int tid = threadIdx.x;
    const double *vk = Vk + (int64_t)ch.prob * c * kMaxK;
    for (int e = tid; e < c * kk; e += kThreads) Vs[e] = vk[e];

    constexpr int EPT = (kMaxK * kMaxK + kThreads - 1) / kThreads;
    double gacc[EPT];
#pragma unroll
    for (int x = 0; x < EPT; ++x) gacc[x] = 0.0;

    const double *Xc = X + ch.x_off;
    double *Yc = Y + ch.y_off;
    for (int r0 = 0; r0 < ch.rows; r0 += PR_RB) {
        const int nr = min(PR_RB, ch.rows - r0);
        __syncthreads();
        for (int e = tid; e < nr * c; e += kThreads) {
            const int rr = e / c, col = e % c;
            Xs[e] = Xc[(int64_t)(r0 + rr) * ld + col];
        }
        __syncthreads();
        for (int e = tid; e < nr * kk; e += kThreads) {
            const int rr = e / kk, j = e % kk;
            double s = 0.0;
            const double *xr = Xs + rr * c;
            for (int a = 0; a < c; ++a) s = fma(xr[a], Vs[a * kk + j], s);
            Ys[e] = s;
            Yc[(int64_t)(r0 + rr) * kk + j] = s;
        }
        __syncthreads();
#pragma unroll
        for (int x = 0; x < EPT; ++x) {
            const int e = tid + x * kThreads;
            if (e < kk * kk) {
                const int a = e / kk, b = e % kk;
                double s = gacc[x];
                for (int rr = 0; rr < nr; ++rr) s = fma(Ys[rr * kk + a], Ys[rr * kk + b], s);
                gacc[x] = s;
            }
        }
    }
    double *G = GYpart + (int64_t)ch.slot * kSlotK;
#pragma unroll
    for (int x = 0; x < EPT; ++x) {
        const int e = tid + x * kThreads;
        if (e < kk * kk) G[e] = gacc[x];
    }
}

__global__ __launch_bounds__(kThreads) void utransform_kernel(double *__restrict__ U, int k,
                                                              const Chunk *__restrict__ chunks,
                                                              const double *__restrict__ F)
{
    constexpr int RB = 32;
    __shared__ double Fs[kMaxK * kMaxK];
    __shared__ double Us[RB * kMaxK];
    const Chunk ch = chunks[blockIdx.x];
    const int tid = threadIdx.x;
    const double *Fp = F + (int64_t)ch.prob * kSlotK;
    for (int e = tid; e < k * k; e += kThreads) Fs[e] = Fp[e];
    double *Uc = U + ch.y_off;
    for (int r0 = 0; r0 < ch.rows; r0 += RB) {
        const int nr = min(RB, ch.rows - r0);
        __syncthreads();
        for (int e = tid; e < nr * k; e += kThreads) Us[e] = Uc[(int64_t)r0 * k + e];
        __syncthreads();
        for (int e = tid; e < nr * k; e += kThreads) {
            const int rr = e / k, j = e % k;
            double s = 0.0;
            for (int l = 0; l < k; ++l) s = fma(Us[rr * k + l], Fs[l * k + j], s);
            Uc[(int64_t)r0 * k + e] = s;
        }
    }
}

}  // namespace

hipError_t launch_project(const double *X, int64_t ld, int c, const Chunk *chunks, int nchunks,
                          const double *Vk, double *Y, double *GYpart, hipStream_t stream)
{
    if (nchunks <= 0) return hipSuccess;
    timing_begin("project", stream);
    const size_t lds = (size_t)(c * kMaxK + PR_RB * c + PR_RB * kMaxK) * sizeof(double);
    static bool attr = false;
    if (!attr) {
        const size_t mx = (size_t)(kMaxC * kMaxK + PR_RB * kMaxC + PR_RB * kMaxK) * sizeof(double);
        hipError_t e = hipFuncSetAttribute((const void *)project_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)mx);
        if (e != hipSuccess) return e;
        attr = true;
    }
    project_kernel<<<nchunks, kThreads, lds, stream>>>(X, ld, c, chunks, Vk, Y, GYpart);
    hipError_t e = hipGetLastError();
    timing_end("project", stream);
    return e;
}

hipError_t launch_utransform(double *U, int k, const Chunk *chunks, int nchunks, const double *F,
                             hipStream_t stream)
{
    if (nchunks <= 0) return hipSuccess;
    timing_begin("utransform", stream);
    utransform_kernel<<<nchunks, kThreads, 0, stream>>>(U, k, chunks, F);
    hipError_t e = hipGetLastError();
    timing_end("utransform", stream);
    return e;
}

}  // namespace zs
