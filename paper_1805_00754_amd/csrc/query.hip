// Query-phase kernels around the stacked SVD (Alg. 2):
//
//  * coef: per touched block, the k x kq factor C_i with
//    U_(S:E) rows of block i = U_(i)[r0:r1) C_i.  For a whole block
//    C_i = U_r(i) (its rows of U_r = Y F); for a boundary block
//    C_i = T_i U_r(i) since U'_i = X U_(i) T_i (Eq. (9) with U' factored).
//    Stored transposed: row j holds column j of C_i, padded with zeros to
//    prod_ld(k) values.
//  * blockprod: the block-diagonal product diag(U'_S, U_(S+1), ..., U'_E) U_r
//    of Eq. (9), one wave per touched block, streaming the block's rows of U
//    from HBM and writing the range's rows of U.  This kernel moves
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
    const int ld = prod_ld(k);
    const double *Tp = pc.t_idx < 0 ? nullptr : T + (int64_t)pc.t_idx * k * k;
    for (int e = tid; e < kq * ld; e += kThreads) {
        const int j = e / ld, l = e % ld;
        double s = 0.0;
        if (l < k) {
            if (Tp == nullptr) {
                s = Ur[l * kq + j];
            } else {
                for (int a = 0; a < k; ++a) s = fma(Tp[l * k + a], Ur[a * kq + j], s);
            }
        }
        Cp[e] = s;
    }
}

// Orders the wave's LDS accesses: everything before it, from every lane, is
// visible to everything after it.  The work-groups of blockprod are one wave.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wave per piece.  Rows go in tiles of 64, one row per lane:
//   1. the tile's rows of U_(i) (contiguous in HBM) are loaded with coalesced
//      8-byte loads, one tile ahead, and copied to LDS unchanged (row stride k);
//   2. each lane takes its row into registers (zero beyond k) and forms its
//      k_q outputs; column j of C_i is KM contiguous values at a wave-uniform
//      address, read through the scalar cache;
//   3. the outputs go back through LDS (row stride k_q) and are written with
//      coalesced stores.
// Every output is sum_l U(r, l) C(l, j) accumulated in l order (the padding
// adds exact zeros).
constexpr int kProdRows = 64;

template <int KM>
__global__ __launch_bounds__(64) void blockprod_kernel(StoreView st, const Piece *__restrict__ pieces,
                                                       const double *__restrict__ C,
                                                       double *__restrict__ Uout)
{
    extern __shared__ __align__(16) double tile[];    // 64 x k
    const Piece pc = pieces[blockIdx.x];
    const int k = st.k;
    const int kq = pc.kq;
    const int lane = threadIdx.x;
    const double *__restrict__ Cp = C + pc.c_off;
    const double *__restrict__ Ub = st.U + (pc.blk * st.b + pc.r0) * k;
    double *__restrict__ out = Uout + pc.out_off;
    const int64_t ldu = pc.ldu;
    const int nrows = pc.r1 - pc.r0;
    const int ntiles = (nrows + kProdRows - 1) / kProdRows;

    double pre[KM];
    {
        const int n = min(kProdRows, nrows) * k;
#pragma unroll
        for (int i = 0; i < KM; ++i) {
            const int e = lane + i * kProdRows;
            pre[i] = (e < n) ? Ub[e] : 0.0;
        }
    }
    for (int t = 0; t < ntiles; ++t) {
        const int row0 = t * kProdRows;
        const int nr = min(kProdRows, nrows - row0);
        wave_sync();                               // the previous tile's outputs are out
#pragma unroll
        for (int i = 0; i < KM; ++i)
            if (i < k) tile[lane + i * kProdRows] = pre[i];
        if (t + 1 < ntiles) {
            const double *Un = Ub + (int64_t)(row0 + kProdRows) * k;
            const int n = min(kProdRows, nrows - row0 - kProdRows) * k;
#pragma unroll
            for (int i = 0; i < KM; ++i) {
                const int e = lane + i * kProdRows;
                if (e < n) pre[i] = Un[e];
            }
        }
        wave_sync();
        double u[KM];
#pragma unroll
        for (int l = 0; l < KM; ++l) u[l] = (l < k) ? tile[lane * k + l] : 0.0;
        wave_sync();                               // every lane holds its row
        if (lane < nr) {
            for (int j = 0; j < kq; ++j) {
                const double *cj = Cp + j * KM;
                double a = 0.0;
#pragma unroll
                for (int l = 0; l < KM; ++l) a = fma(u[l], cj[l], a);
                tile[lane * kq + j] = a;
            }
        }
        wave_sync();
        const int n = nr * kq;
        if (ldu == kq) {                           // the tile is contiguous in the output
            double *o = out + (int64_t)row0 * kq;
#pragma unroll
            for (int i = 0; i < KM; ++i) {
                const int e = lane + i * kProdRows;
                if (i < kq && e < n) o[e] = tile[e];
            }
        } else {
            for (int e = lane; e < n; e += kProdRows) {
                const int r = e / kq;
                out[(int64_t)(row0 + r) * ldu + (e - r * kq)] = tile[e];
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

template <int KM>
hipError_t run_blockprod(StoreView st, const Piece *pieces, int npieces, const double *C, double *U,
                         hipStream_t stream)
{
    const size_t lds = (size_t)kProdRows * st.k * sizeof(double);
    blockprod_kernel<KM><<<npieces, kProdRows, lds, stream>>>(st, pieces, C, U);
    return hipGetLastError();
}

hipError_t launch_blockprod(StoreView st, const Piece *pieces, int npieces, const double *C,
                            double *U, hipStream_t stream)
{
    if (npieces <= 0) return hipSuccess;
    if (st.k < 1 || st.k > kMaxK) return hipErrorInvalidValue;
    timing_begin("blockprod", stream);
    hipError_t e;
    switch (prod_ld(st.k)) {
#define ZS_PROD_CASE(KM) \
    case KM: e = run_blockprod<KM>(st, pieces, npieces, C, U, stream); break;
        ZS_PROD_CASE(4) ZS_PROD_CASE(8) ZS_PROD_CASE(12) ZS_PROD_CASE(16) ZS_PROD_CASE(20)
        ZS_PROD_CASE(24) ZS_PROD_CASE(28) ZS_PROD_CASE(32) ZS_PROD_CASE(48) ZS_PROD_CASE(64)
#undef ZS_PROD_CASE
    default: e = hipErrorInvalidValue;
    }
    timing_end("blockprod", stream);
    return e;
}

}  // namespace zs
