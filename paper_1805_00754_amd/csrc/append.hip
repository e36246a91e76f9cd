// Streaming ingest: rows appended to a store first fill its last block by the
// incremental update of Eqs. (2)-(3), taken for the appended rows at once:
//   [U Sigma V^T; R] = diag(U, I) [Sigma V^T; R],  [Sigma V^T; R] = U' Sigma' V'^T,
//   so the block's new factors are U_new = diag(U, I) U', Sigma', V'.
// These kernels form the stacked rows [Sigma V^T; R] of the last block and the
// product diag(U, I) U'; the SVD in between is the storage phase's own.
#include "zs_internal.h"

namespace zs {
namespace {

// P (k + m1) x c in FP64: rows sigma_j v_j^T of block `blk`, then m1 rows of R.
template <typename TU, typename TR>
__global__ __launch_bounds__(kThreads) void tail_rows_kernel(StoreView st, int64_t blk,
                                                             const TR *__restrict__ R, int64_t ldr,
                                                             int64_t m1, double *__restrict__ P)
{
    const int64_t c = st.c, k = st.k;
    const TU *Vt = static_cast<const TU *>(st.Vt) + blk * k * c;
    for (int64_t e = blockIdx.x * (int64_t)kThreads + threadIdx.x; e < (k + m1) * c;
         e += (int64_t)gridDim.x * kThreads) {
        const int64_t r = e / c, col = e - r * c;
        P[e] = r < k ? st.S[blk * k + r] * (double)Vt[r * c + col]
                     : load_as_double(R, (r - k) * ldr + col);
    }
}

// The last block's new U rows (r_tail + m1 of them, k columns): rows below
// r_tail are U_old U'[0:k, :], the others U'[k + i, :].  FP64 sums in index
// order; stored in the store's element type.
template <typename TU>
__global__ __launch_bounds__(kThreads) void tail_u_kernel(const TU *__restrict__ Uold, int64_t r_tail,
                                                          const TU *__restrict__ Up, int64_t m1, int k,
                                                          TU *__restrict__ Unew)
{
    for (int64_t e = blockIdx.x * (int64_t)kThreads + threadIdx.x; e < (r_tail + m1) * k;
         e += (int64_t)gridDim.x * kThreads) {
        const int64_t i = e / k;
        const int j = (int)(e - i * k);
        double s;
        if (i < r_tail) {
            s = 0.0;
            for (int l = 0; l < k; ++l) s = fma((double)Uold[i * k + l], (double)Up[(int64_t)l * k + j], s);
        } else {
            s = (double)Up[(k + i - r_tail) * k + j];
        }
        Unew[e] = (TU)s;
    }
}

unsigned grid_for(int64_t n)
{
    return (unsigned)std::min<int64_t>((n + kThreads - 1) / kThreads, 65536);
}

template <typename TU>
hipError_t run_tail_rows(StoreView st, int64_t blk, const void *R, int r_type, int64_t ldr,
                         int64_t m1, double *P, hipStream_t stream)
{
    const unsigned g = grid_for((st.k + m1) * st.c);
    if (r_type == kElemF32)
        tail_rows_kernel<TU, float><<<g, kThreads, 0, stream>>>(st, blk, static_cast<const float *>(R), ldr, m1, P);
    else if (r_type == kElemBF16)
        tail_rows_kernel<TU, uint16_t><<<g, kThreads, 0, stream>>>(st, blk, static_cast<const uint16_t *>(R), ldr, m1, P);
    else
        tail_rows_kernel<TU, double><<<g, kThreads, 0, stream>>>(st, blk, static_cast<const double *>(R), ldr, m1, P);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_tail_rows(StoreView st, int64_t blk, const void *R, int r_type, int64_t ldr,
                            int64_t m1, double *P, hipStream_t stream)
{
    return st.f32 ? run_tail_rows<float>(st, blk, R, r_type, ldr, m1, P, stream)
                  : run_tail_rows<double>(st, blk, R, r_type, ldr, m1, P, stream);
}

hipError_t launch_tail_u(const void *Uold, int64_t r_tail, const void *Up, int64_t m1, int k, int f32,
                         void *Unew, hipStream_t stream)
{
    const unsigned g = grid_for((r_tail + m1) * k);
    if (f32)
        tail_u_kernel<float><<<g, kThreads, 0, stream>>>(static_cast<const float *>(Uold), r_tail,
                                                         static_cast<const float *>(Up), m1, k,
                                                         static_cast<float *>(Unew));
    else
        tail_u_kernel<double><<<g, kThreads, 0, stream>>>(static_cast<const double *>(Uold), r_tail,
                                                          static_cast<const double *>(Up), m1, k,
                                                          static_cast<double *>(Unew));
    return hipGetLastError();
}

}  // namespace zs
