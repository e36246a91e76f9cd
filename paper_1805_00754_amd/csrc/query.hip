// Query-phase kernels around the stacked SVD (Alg. 2):
//
//  * coef: per touched block, the k x kq factor C_i with
//    U_(S:E) rows of block i = U_(i)[r0:r1) C_i.  For a whole block
//    C_i = U_r(i) (its rows of U_r = Y F); for a boundary block
//    C_i = T_i U_r(i) since U'_i = X U_(i) T_i (Eq. (9) with U' factored).
//  * blockprod: the block-diagonal product diag(U'_S, U_(S+1), ..., U'_E) U_r
//    of Eq. (9), one work-group per touched block, streaming the block's rows
//    of U from HBM and writing the range's rows of U.  This kernel moves
//    n*k + n*kq values per query and is bound by HBM bandwidth.
#include "zs_internal.h"

namespace zs {
namespace {

__global__ __launch_bounds__(kThreads) void coef_kernel(int k, const Piece *__restrict__ pieces,
                                                        const double *__restrict__ Y,
                                                        const double *__restrict__ F,
                                                        const double *__restrict__ T,
                                                        double *__restrict__ C)
{
    __shared__ double Ur[kMaxK * kMaxK];
    __shared__ double Fs[kMaxK * kMaxK];
    const Piece pc = pieces[blockIdx.x];
    const int kq = pc.kq;
    const int tid = threadIdx.x;
    const double *Fp = F + (int64_t)pc.q * kSlotK;
    for (int e = tid; e < kq * kq; e += kThreads) Fs[e] = Fp[e];
    __syncthreads();
    const double *Yp = Y + pc.y_off;
    for (int e = tid; e < k * kq; e += kThreads) {
        const int l = e / kq, j = e % kq;
        double s = 0.0;
        for (int m = 0; m < kq; ++m) s = fma(Yp[l * kq + m], Fs[m * kq + j], s);
        Ur[e] = s;
    }
    __syncthreads();
    double *Cp = C + pc.c_off;
    if (pc.t_idx < 0) {
        for (int e = tid; e < k * kq; e += kThreads) Cp[e] = Ur[e];
    } else {
        const double *Tp = T + (int64_t)pc.t_idx * k * k;
        for (int e = tid; e < k * kq; e += kThreads) {
            const int l = e / kq, j = e % kq;
            double s = 0.0;
            for (int a = 0; a < k; ++a) s = fma(Tp[l * k + a], Ur[a * kq + j], s);
            Cp[e] = s;
        }
    }
}

// Thread (rl, j) keeps column j of C_i in registers and produces output
// column j for rows rl, rl + NR, ...; U rows are staged through LDS with
// contiguous loads, output rows are written contiguously.
template <int KMAX>
__global__ __launch_bounds__(kThreads) void blockprod_kernel(StoreView st,
                                                             const Piece *__restrict__ pieces,
                                                             const double *__restrict__ C,
                                                             double *__restrict__ Uout)
{
    constexpr int RB = 64;
    __shared__ __align__(16) double Us[RB * KMAX];
    const Piece pc = pieces[blockIdx.x];
    const int k = st.k;
    const int kq = pc.kq;
    const int tid = threadIdx.x;
    const int NR = kThreads / kq;
    const int rl = tid / kq, j = tid % kq;
    const double *Cp = C + pc.c_off;
    double creg[KMAX];
#pragma unroll
    for (int l = 0; l < KMAX; ++l) creg[l] = (l < k && rl < NR) ? Cp[l * kq + j] : 0.0;

    const double *Ub = st.U + (pc.blk * st.b + pc.r0) * k;
    double *out = Uout + pc.out_off;
    const int nrows = pc.r1 - pc.r0;
    for (int r0 = 0; r0 < nrows; r0 += RB) {
        const int nr = min(RB, nrows - r0);
        __syncthreads();
        for (int e = tid; e < nr * k; e += kThreads) Us[e] = Ub[(int64_t)r0 * k + e];
        __syncthreads();
        if (rl < NR) {
            for (int rr = rl; rr < nr; rr += NR) {
                const double *ur = Us + rr * k;
                double acc = 0.0;
#pragma unroll
                for (int l = 0; l < KMAX; ++l)
                    if (l < k) acc = fma(ur[l], creg[l], acc);
                out[(int64_t)(r0 + rr) * pc.ldu + j] = acc;
            }
        }
    }
}

}  // namespace

hipError_t launch_coef(int k, const Piece *pieces, int npieces, const double *Y, const double *F,
                       const double *T, double *C, hipStream_t stream)
{
    if (npieces <= 0) return hipSuccess;
    timing_begin("coef", stream);
    coef_kernel<<<npieces, kThreads, 0, stream>>>(k, pieces, Y, F, T, C);
    hipError_t e = hipGetLastError();
    timing_end("coef", stream);
    return e;
}

hipError_t launch_blockprod(StoreView st, const Piece *pieces, int npieces, const double *C,
                            double *U, hipStream_t stream)
{
    if (npieces <= 0) return hipSuccess;
    timing_begin("blockprod", stream);
    if (st.k <= 16) blockprod_kernel<16><<<npieces, kThreads, 0, stream>>>(st, pieces, C, U);
    else if (st.k <= 32) blockprod_kernel<32><<<npieces, kThreads, 0, stream>>>(st, pieces, C, U);
    else blockprod_kernel<64><<<npieces, kThreads, 0, stream>>>(st, pieces, C, U);
    hipError_t e = hipGetLastError();
    timing_end("blockprod", stream);
    return e;
}

}  // namespace zs
