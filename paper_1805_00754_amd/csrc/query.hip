// Query-phase kernels around the stacked SVD (Alg. 2):
//
//  * coef: per touched block (one work-group per projection chunk), the
//    k x kq factor C_i with
//    U_(S:E) rows of block i = U_(i)[r0:r1) C_i.  For a whole block
//    C_i = U_r(i) (its rows of U_r = Y F); for a boundary block
//    C_i = T_i U_r(i) since U'_i = X U_(i) T_i (Eq. (9) with U' factored).
//    Stored transposed: row j holds column j of C_i, padded with zeros to
//    prod_ld(k) values.
//  * blockprod: the block-diagonal product diag(U'_S, U_(S+1), ..., U'_E) U_r
//    of Eq. (9), one wave per touched block, streaming the block's rows of U
//    and writing the range's rows of U.  This kernel moves n*k + n*kq values
//    per query and is bound by memory bandwidth.
#include "zs_internal.h"

#include <cstdio>

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

__global__ __launch_bounds__(kThreads) void zero_i32_kernel(int32_t *__restrict__ a, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x;
    if (i < n) a[i] = 0;
}

// perm[boff[blk] + rank] = piece, rank taken from a per-block counter.  The
// order of the pieces of one block among themselves does not matter: each
// piece writes its own rows.
__global__ __launch_bounds__(kThreads) void order_pieces_kernel(const Piece *__restrict__ pieces,
                                                                int npieces,
                                                                const int32_t *__restrict__ boff,
                                                                int32_t *__restrict__ bcount,
                                                                int32_t *__restrict__ perm)
{
    const int p = blockIdx.x * kThreads + threadIdx.x;
    if (p >= npieces) return;
    const int64_t blk = pieces[p].blk;
    perm[boff[blk] + atomicAdd(&bcount[blk], 1)] = p;
}

// Y elements per thread carried one piece ahead in coef_kernel (all of Y_i
// while k k_q <= 4 kThreads; the rest is loaded when it is needed).
constexpr int kCoefPre = 4;

// One work-group per chunk of pieces of one query (the projection chunks):
// F (k_q x k_q) is loaded once; per piece, Y_i (k x k_q) gives U_r(i) = Y_i F,
// and C_i = U_r(i) or T_i U_r(i) is written transposed and padded.  The next
// piece's Y_i is loaded into registers while this one is computed.
__global__ __launch_bounds__(kThreads) void coef_kernel(int k, const Piece *__restrict__ pieces,
                                                        const StackChunk *__restrict__ chunks,
                                                        const double *__restrict__ Y,
                                                        const double *__restrict__ F,
                                                        const double *__restrict__ T,
                                                        double *__restrict__ C)
{
    extern __shared__ __align__(16) double sm[];
    const StackChunk ch = chunks[blockIdx.x];
    const int kq = ch.kk;
    const int tid = threadIdx.x;
    const int ld = prod_ld(k);
    double *Fs = sm;                      // kq x kq
    double *Ys = Fs + kq * kq;            // k x kq
    double *Ur = Ys + k * kq;             // k x kq
    double *Ts = Ur + k * kq;             // k x k
    const double *Fp = F + (int64_t)ch.prob * kSlotK;
    for (int e = tid; e < kq * kq; e += kThreads) Fs[e] = Fp[e];
    const int nky = k * kq;
    double ypre[kCoefPre];
    auto fetch = [&](int p) {
        const double *Yn = Y + pieces[ch.piece0 + p].y_off;
#pragma unroll
        for (int x = 0; x < kCoefPre; ++x) {
            const int e = tid + x * kThreads;
            ypre[x] = e < nky ? Yn[e] : 0.0;
        }
    };
    if (ch.npieces > 0) fetch(0);
    for (int p = 0; p < ch.npieces; ++p) {
        const Piece &pc = pieces[ch.piece0 + p];
        const double *Yp = Y + pc.y_off;
        const bool partial = pc.t_idx >= 0;
        __syncthreads();                  // the previous piece is done with Ys, Ur, Ts
#pragma unroll
        for (int x = 0; x < kCoefPre; ++x) {
            const int e = tid + x * kThreads;
            if (e < nky) Ys[e] = ypre[x];
        }
        for (int e = tid + kCoefPre * kThreads; e < nky; e += kThreads) Ys[e] = Yp[e];
        if (partial) {
            const double *Tp = T + (int64_t)pc.t_idx * k * k;
            for (int e = tid; e < k * k; e += kThreads) Ts[e] = Tp[e];
        }
        if (p + 1 < ch.npieces) fetch(p + 1);   // consumed after this piece's products
        __syncthreads();
        // U_r(i) = Y_i F.  From k_q = 17 on in 2 x 2 tiles (rows l0, l0 + 1;
        // columns j0, j0 + 1), where four LDS loads feed four FMAs; below, one
        // output per thread keeps more threads busy.  Either way each output
        // is summed over m in order by one thread (the same bits).
        if (kq < 17) {
            for (int e = tid; e < k * kq; e += kThreads) {
                const int l = e / kq, j = e % kq;
                double s = 0.0;
                for (int m = 0; m < kq; ++m) s = fma(Ys[l * kq + m], Fs[m * kq + j], s);
                Ur[e] = s;
            }
        } else {
            const int ntc = (kq + 1) / 2;
            for (int t = tid; t < ((k + 1) / 2) * ntc; t += kThreads) {
                const int l0 = 2 * (t / ntc), j0 = 2 * (t % ntc);
                const int l1 = min(l0 + 1, k - 1), j1 = min(j0 + 1, kq - 1);
                double s00 = 0.0, s01 = 0.0, s10 = 0.0, s11 = 0.0;
                for (int m = 0; m < kq; ++m) {
                    const double y0 = Ys[l0 * kq + m], y1 = Ys[l1 * kq + m];
                    const double f0 = Fs[m * kq + j0], f1 = Fs[m * kq + j1];
                    s00 = fma(y0, f0, s00);
                    s01 = fma(y0, f1, s01);
                    s10 = fma(y1, f0, s10);
                    s11 = fma(y1, f1, s11);
                }
                Ur[l0 * kq + j0] = s00;
                if (j0 + 1 < kq) Ur[l0 * kq + j0 + 1] = s01;
                if (l0 + 1 < k) {
                    Ur[(l0 + 1) * kq + j0] = s10;
                    if (j0 + 1 < kq) Ur[(l0 + 1) * kq + j0 + 1] = s11;
                }
            }
        }
        __syncthreads();
        double *Cp = C + pc.c_off;
        for (int e = tid; e < kq * ld; e += kThreads) {
            const int j = e / ld, l = e % ld;
            double s = 0.0;
            if (l < k) {
                if (!partial) {
                    s = Ur[l * kq + j];
                } else {
                    for (int a = 0; a < k; ++a) s = fma(Ts[l * k + a], Ur[a * kq + j], s);
                }
            }
            Cp[e] = s;
        }
    }
}

// Orders the wave's LDS accesses: everything before it, from every lane, is
// visible to everything after it (blockprod work-groups are one wave).
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

// Plain stores (aux 0): with the nontemporal hint (aux 2) the product of the
// 1,024-query batch of 320,000-row ranges (52 GB of output) ran 4 % slower.
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, int off, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v),
                                          r, off, 0, 0);
}
__device__ __forceinline__ void buf_store2(__amdgpu_buffer_rsrc_t r, int off, double a, double b)
{
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 v = {a, b};
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), r, off, 0, 0);
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, int off, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}

// Element e of a buffer of TU, as double; the pinned form is volatile (aux bit
// 31) so that the compiler keeps a prefetch where it is written.
template <typename TU, bool PINNED>
__device__ __forceinline__ double buf_elem(__amdgpu_buffer_rsrc_t r, int e)
{
    constexpr int aux = PINNED ? (int)0x80000000u : 0;
    if constexpr (sizeof(TU) == 8)
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, e * 8, 0, aux));
    else
        return (double)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, e * 4, 0, aux));
}

// One wave per piece, rows in tiles of 64 (16 from 48 columns on).  The
// product of a tile with C_i
// runs on the matrix cores (FP64 MFMA 16x16x4): C_i stays in registers for
// the whole piece as B fragments, so the tile loop reads no coefficients.
//   1. the tile's rows of U_(i) (contiguous in HBM) are loaded with coalesced
//      8-byte buffer loads one tile ahead and copied to LDS (from 32
//      columns on with the row stride padded to KM + 1, below);
//   2. A fragments (16 rows x 4 columns) come from LDS; the tile's row
//      blocks times ceil(k_q / 16) column blocks of 16 x 16 accumulators,
//      KM / 4 steps;
//   3. the accumulators go back through LDS (row stride k_q) and are written
//      with coalesced 16-byte stores.
// Operand layout of v_mfma_f64_16x16x4f64 (wave of 64 lanes): A(i, s) in lane
// i + 16 s, B(s, j) in lane j + 16 s, D(i, j) in register i / 4 of lane
// j + 16 (i mod 4).
// Every load and store of the loop is issued unconditionally (the buffer
// range does the bounds check), so the number of memory operations between
// a tile's prefetch and its use is fixed and the wait for the prefetch does
// not also wait for the previous tile's stores.  The prologue issues as many
// dropped 16-byte stores as a tile does to give the first iteration the same
// count; only a tile whose length is not a whole number of 16-byte groups
// adds stores.
// Every output is sum_l U(r, l) C(l, j) over l in order, four terms per
// step; the padding adds exact zeros.
constexpr int kProdRows = 64;
template <int KM> struct ProdRowBlocks { static constexpr int value = KM >= 48 ? 1 : 4; };

// Work-groups are dispatched to the eight XCDs round-robin; work-group w
// takes position (w mod 8) * per + w / 8 of the block-major order, so each
// XCD walks its own contiguous run of blocks and a block's rows of U are
// fetched into one L2 and reused by every query that touches the block.
constexpr int kXcds = 8;

typedef double v4d __attribute__((ext_vector_type(4)));

template <int KM, bool CONTIG, typename TU>
__global__ __launch_bounds__(kProdRows) void blockprod_kernel(StoreView st, const Piece *__restrict__ pieces,
                                                              const int32_t *__restrict__ perm, int npieces,
                                                              const double *__restrict__ C,
                                                              TU *__restrict__ Uout, int xcd)
{
    constexpr int KS = KM / 4;                     // MFMA steps over l
    constexpr int NCB = (KM + 15) / 16;            // 16-column blocks (k_q <= k <= KM)
    // When the last block holds 4 columns (KM = 16 m + 4) it runs on the 4x4x4
    // matrix-core shape: four independent 4 x 4 blocks per instruction at a
    // quarter of the 16x16x4 cost.  Its A operand is the 16x16x4 A fragment
    // unchanged (A(b, i, s) in lane 16 s + 4 b + i); B(s, j) sits in lane
    // 16 s + 4 b + j for every block b, and D(b, i, j) in lane 16 i + 4 b + j.
    constexpr bool TAIL = KM % 16 == 4;
    constexpr int NF = TAIL ? NCB - 1 : NCB;       // full 16-column blocks
    constexpr int NFA = NF > 0 ? NF : 1;
    // From 32 columns on the U tile is stored in LDS at the padded row stride
    // KM + 1 (at a stride of 32 or 64 doubles the 16 rows of an A fragment
    // would share one bank pair); below, at the row stride k of HBM, where
    // the padded form measured slower on the 20-column benchmark batch
    // (12.2 against 10.8 ms: the lower register count gives a third wave per
    // SIMD, which slows the store stream).
    constexpr bool PAD = KM >= 32;
    constexpr int LDT = KM + 1;                    // row stride of the padded U tile
    // Tiles of 64 rows, or of 16 from 48 columns on, where a 64-row tile's
    // prefetch and accumulators would leave one wave per SIMD.
    constexpr int RB = ProdRowBlocks<KM>::value;   // 16-row blocks per tile
    constexpr int TR = 16 * RB;                    // rows per tile
    constexpr int PT = TR * KM / kProdRows;        // tile elements per lane
    extern __shared__ __align__(16) double tile[];    // U tile, then the output tile
    const int per = (npieces + kXcds - 1) / kXcds;
    const int pos = xcd ? (int)(blockIdx.x % kXcds) * per + (int)(blockIdx.x / kXcds) : (int)blockIdx.x;
    if (pos >= npieces) return;
    const Piece pc = pieces[perm[pos]];
    const int k = st.k;
    const int kq = pc.kq;
    const int lane = threadIdx.x;
    const double *__restrict__ Cp = C + pc.c_off;
    // B fragments: B(s, j) = C(4 t + s, 16 cb + j) for step t, zero beyond k_q
    double bf[NFA][KS];
#pragma unroll
    for (int cb = 0; cb < NF; ++cb)
#pragma unroll
        for (int t = 0; t < KS; ++t) {
            const int j = 16 * cb + lane % 16, l = 4 * t + lane / 16;
            bf[cb][t] = j < kq ? Cp[j * KM + l] : 0.0;
        }
    double bt[KS];                                 // tail: B(s, j) = C(4 t + s, 16 NF + j)
#pragma unroll
    for (int t = 0; t < KS; ++t) {
        const int j = 16 * NF + lane % 4, l = 4 * t + lane / 16;
        bt[t] = (TAIL && j < kq) ? Cp[j * KM + l] : 0.0;
    }
    const TU *Ub = static_cast<const TU *>(st.U) + (pc.blk * st.b + pc.r0) * k;
    TU *out = Uout + pc.out_off;
    const int64_t ldu = pc.ldu;
    const int nrows = pc.r1 - pc.r0;
    const int ntiles = (nrows + TR - 1) / TR;
    auto urange = [&](int row0) {
        const int nr = max(0, min(TR, nrows - row0));
        return buf(Ub + (int64_t)row0 * k, nr * k * (int)sizeof(TU));
    };
    // Element e = lane + 64 i of a lane's share of the tile sits in row e / KM
    // and column e mod KM: at e - (e / KM)(KM - k) in HBM (columns past k
    // read past the range, zero) and at e + e / KM in LDS (stride KM + 1).
    const int dk = KM - k;
    auto uoff = [&](int e, int row) { return e - row * KM < k ? e - row * dk : 1 << 27; };

    double pre[PT];
    {
        const __amdgpu_buffer_rsrc_t r = urange(0);
#pragma unroll
        for (int i = 0; i < PT; ++i) {
            const int e = lane + i * kProdRows;
            pre[i] = buf_elem<TU, false>(r, PAD ? uoff(e, e / KM) : e);
        }
        // dropped stores, as many as a tile issues (below)
        const __amdgpu_buffer_rsrc_t none = buf(out, 0);
        if constexpr (CONTIG) {
#pragma unroll
            for (int i = 0; i < PT / (sizeof(TU) == 8 ? 2 : 4); ++i)
                buf_store2(none, (lane + i * kProdRows) * 16, 0.0, 0.0);
        } else {
#pragma unroll
            for (int i = 0; i < PT; ++i) buf_store(none, (lane + i * kProdRows) * (int)sizeof(TU), (TU)0);
        }
    }
    for (int t = 0; t < ntiles; ++t) {
        const int row0 = t * TR;
        const int nr = min(TR, nrows - row0);
        wave_sync();                               // the previous tile's outputs are read
        if constexpr (PAD) {
            // the element positions are recomputed per tile (kept out of
            // registers across tiles)
            int ln = lane;
            asm volatile("" : "+v"(ln));
            const __amdgpu_buffer_rsrc_t r = urange(row0 + TR);   // empty after the last
#pragma unroll
            for (int i = 0; i < PT; ++i) {
                const int e = ln + i * kProdRows, row = e / KM;
                tile[e + row] = pre[i];
                pre[i] = buf_elem<TU, true>(r, uoff(e, row));
            }
        } else {
#pragma unroll
            for (int i = 0; i < PT; ++i) tile[lane + i * kProdRows] = pre[i];
            const __amdgpu_buffer_rsrc_t r = urange(row0 + TR);   // empty after the last
#pragma unroll
            for (int i = 0; i < PT; ++i) pre[i] = buf_elem<TU, true>(r, lane + i * kProdRows);
        }
        wave_sync();
        v4d acc[RB][NFA];
        double acct[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
            for (int cb = 0; cb < NF; ++cb) acc[rb][cb] = (v4d){0.0, 0.0, 0.0, 0.0};
            acct[rb] = 0.0;
#pragma unroll
            for (int s2 = 0; s2 < KS; ++s2) {
                const int col = 4 * s2 + lane / 16;
                double a;
                if constexpr (PAD) {
                    a = tile[(16 * rb + lane % 16) * LDT + col];   // zero past k
                } else {
                    const double x = tile[(16 * rb + lane % 16) * k + col];
                    a = col < k ? x : 0.0;
                }
#pragma unroll
                for (int cb = 0; cb < NF; ++cb)
                    acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bf[cb][s2], acc[rb][cb], 0, 0, 0);
                if constexpr (TAIL)
                    acct[rb] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, bt[s2], acct[rb], 0, 0, 0);
            }
        }
        wave_sync();                               // every lane has read its A fragments
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
            for (int cb = 0; cb < NF; ++cb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int row = 16 * rb + 4 * v + lane / 16, col = 16 * cb + lane % 16;
                    if (col < kq) tile[row * kq + col] = acc[rb][cb][v];
                }
            if constexpr (TAIL) {
                const int row = 16 * rb + 4 * ((lane % 16) / 4) + lane / 16, col = 16 * NF + lane % 4;
                if (col < kq) tile[row * kq + col] = acct[rb];
            }
        }
        wave_sync();
        if (CONTIG) {                              // the tile is contiguous in the output
            const __amdgpu_buffer_rsrc_t r = buf(out + (int64_t)row0 * kq, nr * kq * (int)sizeof(TU));
            if constexpr (sizeof(TU) == 8) {
                // 16-byte stores of consecutive output pairs (1.06x faster
                // than 8-byte stores on the benchmark batch).  A pair that
                // straddles the end of an odd-length tile is stored again as
                // its in-range element, whatever the range check does with
                // the half past the end.
#pragma unroll
                for (int i = 0; i < PT / 2; ++i) {
                    const int e = 2 * (lane + i * kProdRows);
                    buf_store2(r, e * 8, tile[e], tile[e + 1]);
                }
                const int n = nr * kq;
                if (n & 1) buf_store(r, (n - 1) * 8, tile[n - 1]);
            } else {
                // FP32 outputs in 16-byte quads, a straddling quad again
                // element by element
                typedef float f4 __attribute__((ext_vector_type(4)));
                typedef unsigned u4 __attribute__((ext_vector_type(4)));
#pragma unroll
                for (int i = 0; i < PT / 4; ++i) {
                    const int e = 4 * (lane + i * kProdRows);
                    const f4 q = {(float)tile[e], (float)tile[e + 1], (float)tile[e + 2], (float)tile[e + 3]};
                    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, q), r, e * 4, 0, 0);
                }
                const int n = nr * kq;
                for (int e = n & ~3; e < n; ++e) buf_store(r, e * 4, (float)tile[e]);
            }
        } else {
            const int n = nr * kq;
            for (int e = lane; e < n; e += kProdRows) {
                const int rr = e / kq;
                out[(int64_t)(row0 + rr) * ldu + (e - rr * kq)] = (TU)tile[e];
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

hipError_t launch_coef(int k, int kq_max, const Piece *pieces, const StackChunk *chunks,
                       int nchunks, const double *Y, const double *F, const double *T, double *C,
                       hipStream_t stream)
{
    if (nchunks <= 0) return hipSuccess;
    const size_t lds = (size_t)(kq_max * kq_max + 2 * k * kq_max + k * k) * sizeof(double);
    static size_t cur = 0;
    {
        hipError_t e = ensure_lds((const void *)coef_kernel, lds, cur);
        if (e != hipSuccess) return e;
    }
    timing_begin("coef", stream);
    coef_kernel<<<nchunks, kThreads, lds, stream>>>(k, pieces, chunks, Y, F, T, C);
    hipError_t e = hipGetLastError();
    timing_end("coef", stream);
    return e;
}

// Work order: block-major positions dealt to the XCDs in runs (0) or in
// dispatch order (1); each piece's outputs are the same bits either way, so
// the autotuner picks per shape.
template <int KM, typename TU>
hipError_t run_blockprod(StoreView st, const Piece *pieces, const int32_t *perm, int npieces,
                         const double *C, void *U, bool contiguous, hipStream_t stream)
{
    const size_t lds = (size_t)16 * ProdRowBlocks<KM>::value * (KM >= 32 ? KM + 1 : KM) * sizeof(double);
    const unsigned grid = (unsigned)(kXcds * ((npieces + kXcds - 1) / kXcds));
    TU *out = static_cast<TU *>(U);
    char key[80];
    snprintf(key, sizeof key, "k=%d f32=%d contig=%d n=%d", st.k, (int)(sizeof(TU) == 4),
             (int)contiguous, tune_bucket(npieces));
    return tuned_launch("blockprod_order", key, 2, 0, stream, [&](int v) {
        const int xcd = v == 0 ? 1 : 0;
        if (contiguous)
            blockprod_kernel<KM, true, TU><<<grid, kProdRows, lds, stream>>>(st, pieces, perm, npieces, C,
                                                                           out, xcd);
        else
            blockprod_kernel<KM, false, TU><<<grid, kProdRows, lds, stream>>>(st, pieces, perm, npieces, C,
                                                                            out, xcd);
        return hipGetLastError();
    });
}

hipError_t launch_order_pieces(const Piece *pieces, int npieces, int64_t nb, const int32_t *boff,
                               int32_t *bcount, int32_t *perm, hipStream_t stream)
{
    if (npieces <= 0) return hipSuccess;
    timing_begin("order", stream);
    zero_i32_kernel<<<(unsigned)((nb + kThreads - 1) / kThreads), kThreads, 0, stream>>>(bcount, nb);
    order_pieces_kernel<<<(unsigned)((npieces + kThreads - 1) / kThreads), kThreads, 0, stream>>>(
        pieces, npieces, boff, bcount, perm);
    hipError_t e = hipGetLastError();
    timing_end("order", stream);
    return e;
}

hipError_t launch_blockprod(StoreView st, const Piece *pieces, const int32_t *perm, int npieces,
                            const double *C, void *U, bool contiguous, hipStream_t stream)
{
    if (npieces <= 0) return hipSuccess;
    if (st.k < 1 || st.k > kMaxK) return hipErrorInvalidValue;
    timing_begin("blockprod", stream);
    hipError_t e;
    switch (prod_ld(st.k)) {
#define ZS_PROD_CASE(KM) \
    case KM:                                                                                    \
        e = st.f32 ? run_blockprod<KM, float>(st, pieces, perm, npieces, C, U, contiguous, stream)  \
                   : run_blockprod<KM, double>(st, pieces, perm, npieces, C, U, contiguous, stream); \
        break;
        ZS_PROD_CASE(4) ZS_PROD_CASE(8) ZS_PROD_CASE(12) ZS_PROD_CASE(16) ZS_PROD_CASE(20)
        ZS_PROD_CASE(24) ZS_PROD_CASE(28) ZS_PROD_CASE(32) ZS_PROD_CASE(48) ZS_PROD_CASE(64)
#undef ZS_PROD_CASE
    default: e = hipErrorInvalidValue;
    }
    timing_end("blockprod", stream);
    return e;
}

}  // namespace zs
