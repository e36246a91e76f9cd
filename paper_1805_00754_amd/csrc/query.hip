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

// Pieces of every query from its descriptor: piece p of query q is block
// S + p, rows [lo, rows) for the first, [0, hi) for the last (Alg. 3 index
// math), with its offsets in Y, C and the caller's U.
__global__ __launch_bounds__(kThreads) void expand_pieces_kernel(StoreView st,
                                                                 const QueryDesc *__restrict__ qd,
                                                                 Piece *__restrict__ pieces)
{
    const QueryDesc d = qd[blockIdx.y];
    const int p = blockIdx.x * kThreads + threadIdx.x;
    if (p >= d.np) return;
    const int64_t blk = d.S + p;
    const int64_t rows = min(st.b, st.t - blk * st.b);
    Piece pc;
    pc.blk = blk;
    pc.r0 = p == 0 ? d.lo : 0;
    pc.r1 = p == d.np - 1 ? d.hi : (int32_t)rows;
    pc.y_off = d.y0 + (int64_t)p * st.k * d.kq;
    pc.c_off = d.c0 + (int64_t)p * prod_ld(st.k) * d.kq;
    pc.out_off = d.u_off + (blk * st.b + pc.r0 - d.ts) * d.ldu;
    pc.ldu = d.ldu;
    pc.q = blockIdx.y;
    pc.kq = d.kq;
    const bool partial = pc.r0 != 0 || pc.r1 != rows;
    pc.t_idx = partial ? d.t0 + (p == 0 ? 0 : d.first_partial) : -1;
    pc.pad = 0;
    pieces[d.piece0 + p] = pc;
}

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

// Buffer resource over `bytes` bytes at `p`: loads beyond the range return
// zero and stores beyond it are dropped, so the tile loops need no guards
// (raw buffer, dword format word of the gfx9 family).
// Its arguments are wave-uniform; readfirstlane says so to the compiler.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf(const void *p, int bytes)
{
    const uint64_t a = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    void *q = reinterpret_cast<void *>(((uint64_t)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(q, 0, __builtin_amdgcn_readfirstlane(bytes), 0x00020000);
}

__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, int off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

// aux 2: nontemporal; the output is written once and not read back here
__device__ __forceinline__ void buf_store_nt(__amdgpu_buffer_rsrc_t r, int off, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v),
                                          r, off, 0, 2);
}

// One wave per piece.  Rows go in tiles of 64, one row per lane:
//   1. the tile's rows of U_(i) (contiguous in HBM) are loaded with coalesced
//      8-byte buffer loads one tile ahead, and copied to LDS unchanged;
//   2. each lane takes its row into registers (zero beyond k) and forms its
//      k_q outputs; column j of C_i is KM contiguous values at a wave-uniform
//      address, read through the scalar cache;
//   3. the outputs go back through LDS (row stride k_q) and are written with
//      coalesced nontemporal stores.
// Every load and store of the loop is issued unconditionally (the buffer
// range does the bounds check), so the number of memory operations between
// a tile's prefetch and its use is fixed and the wait for the prefetch does
// not also wait for the previous tile's stores.  The prologue issues KM
// dropped stores to give the first iteration the same count.
// Every output is sum_l U(r, l) C(l, j) accumulated in l order (the padding
// adds exact zeros).
constexpr int kProdRows = 64;

template <int KM, bool CONTIG>
__global__ __launch_bounds__(64) void blockprod_kernel(StoreView st, const Piece *__restrict__ pieces,
                                                       const double *__restrict__ C,
                                                       double *__restrict__ Uout)
{
    extern __shared__ __align__(16) double tile[];    // 64 x KM
    const Piece pc = pieces[blockIdx.x];
    const int k = st.k;
    const int kq = pc.kq;
    const int lane = threadIdx.x;
    const double *__restrict__ Cp = C + pc.c_off;
    const double *Ub = st.U + (pc.blk * st.b + pc.r0) * k;
    double *out = Uout + pc.out_off;
    const int64_t ldu = pc.ldu;
    const int nrows = pc.r1 - pc.r0;
    const int ntiles = (nrows + kProdRows - 1) / kProdRows;
    auto urange = [&](int row0) {
        const int nr = max(0, min(kProdRows, nrows - row0));
        return buf(Ub + (int64_t)row0 * k, nr * k * (int)sizeof(double));
    };

    double pre[KM];
    {
        const __amdgpu_buffer_rsrc_t r = urange(0);
#pragma unroll
        for (int i = 0; i < KM; ++i) pre[i] = buf_load(r, (lane + i * kProdRows) * 8);
        const __amdgpu_buffer_rsrc_t none = buf(out, 0);
#pragma unroll
        for (int i = 0; i < KM; ++i) buf_store_nt(none, (lane + i * kProdRows) * 8, 0.0);
    }
    for (int t = 0; t < ntiles; ++t) {
        const int row0 = t * kProdRows;
        const int nr = min(kProdRows, nrows - row0);
        wave_sync();                               // the previous tile's outputs are read
#pragma unroll
        for (int i = 0; i < KM; ++i) tile[lane + i * kProdRows] = pre[i];
        {
            const __amdgpu_buffer_rsrc_t r = urange(row0 + kProdRows);   // empty after the last
#pragma unroll
            for (int i = 0; i < KM; ++i) pre[i] = buf_load(r, (lane + i * kProdRows) * 8);
        }
        wave_sync();
        double u[KM];
#pragma unroll
        for (int l = 0; l < KM; ++l) {
            const double x = tile[lane * k + l];
            u[l] = (l < k) ? x : 0.0;
        }
        wave_sync();                               // every lane holds its row
        for (int j = 0; j < kq; ++j) {
            const double *cj = Cp + j * KM;
            double a = 0.0;
#pragma unroll
            for (int l = 0; l < KM; ++l) a = fma(u[l], cj[l], a);
            tile[lane * kq + j] = a;
        }
        wave_sync();
        if (CONTIG) {                              // the tile is contiguous in the output
            const __amdgpu_buffer_rsrc_t r = buf(out + (int64_t)row0 * kq, nr * kq * (int)sizeof(double));
#pragma unroll
            for (int i = 0; i < KM; ++i)
                buf_store_nt(r, (lane + i * kProdRows) * 8, tile[lane + i * kProdRows]);
        } else {
            const int n = nr * kq;
            for (int e = lane; e < n; e += kProdRows) {
                const int rr = e / kq;
                out[(int64_t)(row0 + rr) * ldu + (e - rr * kq)] = tile[e];
            }
        }
    }
}

}  // namespace

hipError_t launch_expand_pieces(StoreView st, const QueryDesc *qd, int nq, int max_np, Piece *pieces,
                                hipStream_t stream)
{
    if (nq <= 0 || max_np <= 0) return hipSuccess;
    timing_begin("expand", stream);
    const dim3 grid((unsigned)((max_np + kThreads - 1) / kThreads), (unsigned)nq);
    expand_pieces_kernel<<<grid, kThreads, 0, stream>>>(st, qd, pieces);
    hipError_t e = hipGetLastError();
    timing_end("expand", stream);
    return e;
}

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
                         bool contiguous, hipStream_t stream)
{
    const size_t lds = (size_t)kProdRows * KM * sizeof(double);
    if (contiguous)
        blockprod_kernel<KM, true><<<npieces, kProdRows, lds, stream>>>(st, pieces, C, U);
    else
        blockprod_kernel<KM, false><<<npieces, kProdRows, lds, stream>>>(st, pieces, C, U);
    return hipGetLastError();
}

hipError_t launch_blockprod(StoreView st, const Piece *pieces, int npieces, const double *C,
                            double *U, bool contiguous, hipStream_t stream)
{
    if (npieces <= 0) return hipSuccess;
    if (st.k < 1 || st.k > kMaxK) return hipErrorInvalidValue;
    timing_begin("blockprod", stream);
    hipError_t e;
    switch (prod_ld(st.k)) {
#define ZS_PROD_CASE(KM) \
    case KM: e = run_blockprod<KM>(st, pieces, npieces, C, U, contiguous, stream); break;
        ZS_PROD_CASE(4) ZS_PROD_CASE(8) ZS_PROD_CASE(12) ZS_PROD_CASE(16) ZS_PROD_CASE(20)
        ZS_PROD_CASE(24) ZS_PROD_CASE(28) ZS_PROD_CASE(32) ZS_PROD_CASE(48) ZS_PROD_CASE(64)
#undef ZS_PROD_CASE
    default: e = hipErrorInvalidValue;
    }
    timing_end("blockprod", stream);
    return e;
}

}  // namespace zs
