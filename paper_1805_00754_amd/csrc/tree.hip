// Gram tree of the stored blocks.
//
// The stacked matrix of a query (Alg. 2) holds the rows Sigma_(i) V_(i)^T
// of every whole block in the range, so its Gram M^T M contains
// sum_i V_(i) Sigma_(i)^2 V_(i)^T over those blocks.  The storage phase keeps
// these c x c block Grams in a binary tree over the blocks (leaf i = block i,
// inner node = sum of its two children, leaves padded to a power of two);
// a query then assembles the whole-block part of its Gram from at most
// 2 log2(nb) nodes instead of touching all K stack rows.  Every node is a sum
// of positive semi-definite terms, so no cancellation occurs.
#include "zs_internal.h"

#include <algorithm>

namespace zs {
namespace {

// leaf i: sum_j sigma_ij^2 v_ij v_ij^T  (zero beyond the last block)
template <typename TU>
__global__ __launch_bounds__(kThreads) void leaf_gram_kernel(StoreView st, int64_t nleaves,
                                                             double *__restrict__ tree,
                                                             int64_t leaf0)
{
    extern __shared__ __align__(16) double Ws[];   // k x c rows sigma_j v_j^T
    const int64_t i = blockIdx.x;
    const int c = (int)st.c, k = st.k;
    const int64_t nb = (st.t + st.b - 1) / st.b;
    double *G = tree + (leaf0 + i) * c * c;
    const int tid = threadIdx.x;
    if (i >= nb) {
        for (int e = tid; e < c * c; e += kThreads) G[e] = 0.0;
        return;
    }
    const TU *Vt = static_cast<const TU *>(st.Vt) + i * k * c;
    for (int e = tid; e < k * c; e += kThreads) Ws[e] = (double)Vt[e] * st.S[i * k + e / c];
    __syncthreads();
    for (int e = tid; e < c * c; e += kThreads) {
        const int a = e / c, b = e % c;
        double s = 0.0;
        for (int j = 0; j < k; ++j) s = fma(Ws[j * c + a], Ws[j * c + b], s);
        G[e] = s;
    }
    (void)nleaves;
}

// nodes [node0, node0 + nnodes): node p = node 2p + node 2p+1
__global__ __launch_bounds__(kThreads) void tree_level_kernel(int c, double *__restrict__ tree,
                                                              int64_t node0)
{
    const int64_t p = node0 + blockIdx.y;
    const int64_t cc = (int64_t)c * c;
    const double *L = tree + 2 * p * cc;
    const double *R = tree + (2 * p + 1) * cc;
    double *D = tree + p * cc;
    for (int64_t e = blockIdx.x * (int64_t)kThreads + threadIdx.x; e < cc;
         e += (int64_t)gridDim.x * kThreads)
        D[e] = L[e] + R[e];
}

// Rows sigma_ij v_ij^T of every block in FP64 (the input of the Gram kernel
// when c is too large for one work-group's LDS), and zero leaves past nb.
template <typename TU>
__global__ __launch_bounds__(kThreads) void scale_rows_kernel(StoreView st, int64_t nb,
                                                              double *__restrict__ rows)
{
    const int64_t kc = (int64_t)st.k * st.c;
    const TU *Vt = static_cast<const TU *>(st.Vt);
    for (int64_t e = blockIdx.x * (int64_t)kThreads + threadIdx.x; e < nb * kc;
         e += (int64_t)gridDim.x * kThreads)
        rows[e] = (double)Vt[e] * st.S[e / st.c];
}

__global__ __launch_bounds__(kThreads) void zero_kernel(double *__restrict__ p, int64_t n)
{
    for (int64_t e = blockIdx.x * (int64_t)kThreads + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * kThreads)
        p[e] = 0.0;
}

}  // namespace

hipError_t launch_scale_rows(StoreView st, int64_t nb, double *rows, hipStream_t stream)
{
    const int64_t n = nb * st.k * st.c;
    const unsigned grid = (unsigned)std::min<int64_t>((n + kThreads - 1) / kThreads, 65536);
    if (st.f32)
        scale_rows_kernel<float><<<grid, kThreads, 0, stream>>>(st, nb, rows);
    else
        scale_rows_kernel<double><<<grid, kThreads, 0, stream>>>(st, nb, rows);
    return hipGetLastError();
}

hipError_t launch_zero(double *p, int64_t n, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const unsigned grid = (unsigned)std::min<int64_t>((n + kThreads - 1) / kThreads, 65536);
    zero_kernel<<<grid, kThreads, 0, stream>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_leaf_gram(StoreView st, int64_t nleaves, double *tree, int64_t leaf0,
                            hipStream_t stream)
{
    if (nleaves <= 0) return hipSuccess;
    const size_t lds = (size_t)st.k * st.c * sizeof(double);
    static size_t cur_f = 0, cur_d = 0;   // one limit per instantiation
    {
        hipError_t e = st.f32 ? ensure_lds((const void *)leaf_gram_kernel<float>, lds, cur_f)
                              : ensure_lds((const void *)leaf_gram_kernel<double>, lds, cur_d);
        if (e != hipSuccess) return e;
    }
    timing_begin("leaf_gram", stream);
    if (st.f32)
        leaf_gram_kernel<float><<<(unsigned)nleaves, kThreads, lds, stream>>>(st, nleaves, tree, leaf0);
    else
        leaf_gram_kernel<double><<<(unsigned)nleaves, kThreads, lds, stream>>>(st, nleaves, tree, leaf0);
    hipError_t e = hipGetLastError();
    timing_end("leaf_gram", stream);
    return e;
}

hipError_t launch_tree_level(int c, double *tree, int64_t node0, int64_t nnodes,
                             hipStream_t stream)
{
    if (nnodes <= 0) return hipSuccess;
    timing_begin("tree_level", stream);
    const int64_t cc = (int64_t)c * c;
    const unsigned gx = (unsigned)((cc + 4 * kThreads - 1) / (4 * kThreads));
    tree_level_kernel<<<dim3(gx, (unsigned)nnodes), kThreads, 0, stream>>>(c, tree, node0);
    hipError_t e = hipGetLastError();
    timing_end("tree_level", stream);
    return e;
}

}  // namespace zs
