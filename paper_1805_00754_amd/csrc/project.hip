// Projection of the data on the first-stage eigenvectors, and the in-place
// U formation of the storage phase.
//
//  * project: for a chunk of rows of a block of A, Y = X V_k (rows x kk,
//    written out) and the partial Gram Y^T Y (kk x kk, one slot per chunk).
//  * stack_project: the same for a query's stacked matrix M, whose rows are
//    read where they live: Sigma_(i) V_(i)^T rows of the store for whole
//    blocks, the Partial-SVD rows for boundary blocks (the stack of Alg. 2).  M is
//    never materialised.
//  * utransform: U_(i) <- Y_(i) F_(i) in place (F = W Sigma^-1 with the sign
//    rule folded in), giving the block's left singular vectors.
//
// project and stack_project share one tile body (one wave per chunk, tiles of
// 32 or 64 rows), described at tile_project.
#include <cstdio>

#include "zs_internal.h"

namespace zs {
namespace {

// Orders the wave's LDS accesses (stack_project work-groups are one wave).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// tile_project: one wave per chunk, tiles of 16 RBN rows (RBN = 2 row blocks
// for 16 < kq <= 32, which keeps two waves per SIMD without spills; 4 else).
// Row r of a tile is s_r x_r for a row x_r in HBM and a scale s_r (the
// caller's row function gives both, and the row's element type).  The tile
// product X V_k runs on the matrix cores (FP64 MFMA 16x16x4) over 16-column
// panels, RBN row blocks times ceil(kq / 16) column blocks; each lane loads its A fragments (four
// consecutive columns of one row each) straight from HBM one panel ahead of
// the matrix-core work, and the B fragments of V_k from cache.  Operand layout: A(i, s)
// in lane i + 16 s, B(s, j) in lane j + 16 s, D(i, j) in register i / 4 of
// lane j + 16 (i mod 4).  The scaled tile Y = S X V_k goes out through LDS with
// coalesced stores.  Its Gram Y^T Y is accumulated on the matrix cores
// straight from the D fragments: register v of block (rb, cb) holds
// Y(16 rb + 4 v + s, 16 cb + i) in lane i + 16 s, which is the A layout of
// (Y^T)(16 cb + i, s) and the B layout of Y(s, 16 cb' + j), so each pair of
// column blocks takes 16 MFMAs per tile and no LDS traffic.
constexpr int kPanel = 16;
typedef double v4d __attribute__((ext_vector_type(4)));
typedef const double __attribute__((address_space(1))) gdouble;
typedef const float __attribute__((address_space(1))) gfloat;
typedef const uint16_t __attribute__((address_space(1))) gushort;
// vectors of consecutive row elements; rows are only element-aligned
typedef double dbl2 __attribute__((ext_vector_type(2)));
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef uint16_t ush4 __attribute__((ext_vector_type(4)));
typedef const dbl2 __attribute__((address_space(1), aligned(8))) gdouble2;
typedef const flt4 __attribute__((address_space(1), aligned(4))) gfloat4;
typedef const ush4 __attribute__((address_space(1), aligned(2))) gushort4;

// A row of a tile: where it starts, its element type (ElemType) and its scale.
struct RowRef {
    const char *p;
    int type;
    double scale;
};

__device__ __forceinline__ double row_elem(const char *p, int type, int i)
{
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    if (type == kElemF64) return reinterpret_cast<const gdouble *>(a)[i];
    if (type == kElemF32) return (double)reinterpret_cast<const gfloat *>(a)[i];
    return (double)__uint_as_float((uint32_t)reinterpret_cast<const gushort *>(a)[i] << 16);
}

// Rows of one element type known at compile time (kMixed: per row, at run time).
constexpr int kMixed = -1;

template <int TYPE>
__device__ __forceinline__ double typed_elem(const char *p, int type, int i)
{
    const uintptr_t a = reinterpret_cast<uintptr_t>(p);
    if constexpr (TYPE == kElemF64) return reinterpret_cast<const gdouble *>(a)[i];
    else if constexpr (TYPE == kElemF32) return (double)reinterpret_cast<const gfloat *>(a)[i];
    else if constexpr (TYPE == kElemBF16)
        return (double)__uint_as_float((uint32_t)reinterpret_cast<const gushort *>(a)[i] << 16);
    else return row_elem(p, type, i);
}

// rows rows of the chunk (row r from row(r)), V_k c x kq row-major; Y rows of
// kq values from Yout, the kq x kq Gram to G.  sm holds 64 x max(17, kq + 1).
template <int KQM, int TYPE, class RowFn>
__device__ __forceinline__ void tile_project(const RowFn &row, int rows, int c, int kq,
                                             const double *__restrict__ V, double *__restrict__ Yout,
                                             double *__restrict__ G, RowRef fallback, double *sm)
{
    constexpr int NCB = (KQM + 15) / 16;           // 16-column blocks of Y
    // With KQM = 16 m + 4 (m >= 1) the last block has 4 columns and runs on
    // the 4x4x4 matrix-core shape at a quarter of the cost: its A operand is
    // the 16x16x4 A fragment unchanged (A(b, i, s) in lane 16 s + 4 b + i),
    // B(s, j) sits in lane 16 s + 4 b + j for every block b, and D(b, i, j)
    // in lane 16 i + 4 b + j.  The result is moved into the 16 x 16 layout of
    // the last block afterwards, so the rest of the tile does not change.
    constexpr bool TAIL = KQM > 16 && KQM % 16 == 4;
    constexpr int NF = TAIL ? NCB - 1 : NCB;       // blocks on the 16x16x4 shape
    constexpr int RBN = (KQM > 16 && KQM <= 32) ? 2 : 4;   // 16-row blocks per tile
    constexpr int TR = 16 * RBN;                   // rows per tile
    const int lane = threadIdx.x;
    const int ldy = kq + 1;
    v4d gacc[NCB][NCB];
#pragma unroll
    for (int ci = 0; ci < NCB; ++ci)
#pragma unroll
        for (int cj = 0; cj < NCB; ++cj) gacc[ci][cj] = (v4d){0.0, 0.0, 0.0, 0.0};

    for (int r0 = 0; r0 < rows; r0 += TR) {
        const int nr = min(TR, rows - r0);
        // lanes past the tile read the fallback row with scale 0
        const RowRef rr = lane < nr ? row(r0 + lane) : fallback;
        const double scale = lane < nr ? rr.scale : 0.0;
        v4d acc[RBN][NCB];
        double acct[RBN];                          // the 4-column block (TAIL)
#pragma unroll
        for (int rb = 0; rb < RBN; ++rb) {
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = (v4d){0.0, 0.0, 0.0, 0.0};
            acct[rb] = 0.0;
        }
        // A fragment (rb, t) of a panel is X(16 rb + i, a0 + 4 t + s) in lane
        // i + 16 s: the lane reads row 16 rb + lane % 16 itself, whose start
        // and type it takes from the row's owner lane once per tile.
        const char *rp[RBN];
        int rt[RBN];
        {
            const uint64_t pa = reinterpret_cast<uint64_t>(rr.p);
#pragma unroll
            for (int rb = 0; rb < RBN; ++rb) {
                const int owner = 16 * rb + lane % 16;
                const uint32_t lo = __shfl((uint32_t)pa, owner, 64);
                const uint32_t hi = __shfl((uint32_t)(pa >> 32), owner, 64);
                rp[rb] = reinterpret_cast<const char *>(((uint64_t)hi << 32) | lo);
                rt[rb] = __shfl(rr.type, owner, 64);
            }
        }
        const int sc4 = lane / 16;
        // A fragments of the panel at a0 (from HBM), and its B fragments (from
        // cache).  MFMA t of a panel takes panel column kcol(t, s) as its
        // contraction index s: the order of the 16 columns over the four
        // MFMAs is free as long as A and B agree, and this one gives each lane
        // four consecutive columns of its row, so that without CLAMP (c a
        // multiple of the panel width) a lane reads its row's part of a panel
        // with 16-byte loads (two for FP64, one for FP32, one 8-byte for BF16).
        // With CLAMP every element load is issued at a clamped address: no
        // load sits under a branch, so the wait for a panel does not also wait
        // for the next one.  Past column c the A fragments repeat column c - 1,
        // a real element, and meet rows of B that are zeroed by an exact
        // multiply.
        // (one order for every element type: FP32 or BF16 input widened to
        // FP64 gives the same sums, bit for bit, as the widened input itself)
        auto kcol = [&](int t) { return 4 * sc4 + t; };
        auto load_a = [&](auto clamp, int a0, double (&af)[RBN][4]) {
            if constexpr (!decltype(clamp)::value && TYPE != kMixed) {
#pragma unroll
                for (int rb = 0; rb < RBN; ++rb) {
                    const uintptr_t ra = reinterpret_cast<uintptr_t>(rp[rb]);
                    if constexpr (TYPE == kElemF64) {
                        const gdouble2 *q = reinterpret_cast<const gdouble2 *>(ra + 8 * (a0 + 4 * sc4));
                        const dbl2 lo = q[0], hi = q[1];
                        af[rb][0] = lo.x;
                        af[rb][1] = lo.y;
                        af[rb][2] = hi.x;
                        af[rb][3] = hi.y;
                    } else if constexpr (TYPE == kElemF32) {
                        const flt4 v = *reinterpret_cast<const gfloat4 *>(ra + 4 * (a0 + 4 * sc4));
                        af[rb][0] = v.x;
                        af[rb][1] = v.y;
                        af[rb][2] = v.z;
                        af[rb][3] = v.w;
                    } else {
                        const ush4 v = *reinterpret_cast<const gushort4 *>(ra + 2 * (a0 + 4 * sc4));
                        af[rb][0] = __uint_as_float((uint32_t)v.x << 16);
                        af[rb][1] = __uint_as_float((uint32_t)v.y << 16);
                        af[rb][2] = __uint_as_float((uint32_t)v.z << 16);
                        af[rb][3] = __uint_as_float((uint32_t)v.w << 16);
                    }
                }
            } else {
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int col = a0 + kcol(t);
                    const int colc = decltype(clamp)::value ? min(col, c - 1) : col;
#pragma unroll
                    for (int rb = 0; rb < RBN; ++rb) af[rb][t] = typed_elem<TYPE>(rp[rb], rt[rb], colc);
                }
            }
        };
        // column of B this lane holds in block cb (the 4x4x4 tail: lane % 4)
        auto bcol = [&](int cb) { return (TAIL && cb == NF) ? 16 * NF + lane % 4 : 16 * cb + lane % 16; };
        auto load_b = [&](int a0, double (&bq)[NCB][4]) {
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    bq[cb][t] = V[min(a0 + kcol(t), c - 1) * kq + min(bcol(cb), kq - 1)];
        };
        // the products of one panel: its B fragments are loaded here (from
        // cache), after the loads already in flight, and their rows past c and
        // columns past kq are zeroed by an exact multiply
        auto panel = [&](int a0, const double (&af)[RBN][4]) {
            double bf[NCB][4];
            load_b(a0, bf);
            if constexpr (KQM <= 32) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    bf[cb][t] *= (a0 + kcol(t) < c && bcol(cb) < kq) ? 1.0 : 0.0;
#pragma unroll
            for (int rb = 0; rb < RBN; ++rb)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
#pragma unroll
                    for (int cb = 0; cb < NF; ++cb)
                        acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[rb][t], bf[cb][t], acc[rb][cb], 0, 0, 0);
                    if constexpr (TAIL)
                        acct[rb] = __builtin_amdgcn_mfma_f64_4x4x4f64(af[rb][t], bf[NF][t], acct[rb], 0, 0, 0);
                }
        };
        auto panels = [&](auto clamp) {
            if constexpr (KQM <= 32) {
                // two sets of A registers in turn: the next panel's A loads are
                // in flight during this panel's products, and no register copy
                // between the sets waits for them
                double a1[RBN][4], a2[RBN][4];
                load_a(clamp, 0, a1);
                for (int a0 = 0; a0 < c; a0 += 2 * kPanel) {
                    // past c: a clamped panel that is not used, or none
                    if (decltype(clamp)::value || a0 + kPanel < c) load_a(clamp, a0 + kPanel, a2);
                    __builtin_amdgcn_sched_barrier(0);
                    panel(a0, a1);
                    if (a0 + kPanel >= c) break;
                    if (decltype(clamp)::value || a0 + 2 * kPanel < c) load_a(clamp, a0 + 2 * kPanel, a1);
                    __builtin_amdgcn_sched_barrier(0);
                    panel(a0 + kPanel, a2);
                }
            } else {
                // wider tiles have no registers to spare for a second set
                for (int a0 = 0; a0 < c; a0 += kPanel) {
                    double af[RBN][4];
                    load_a(clamp, a0, af);
                    panel(a0, af);
                }
            }
        };
        if (c % kPanel == 0)
            panels(std::false_type{});
        else
            panels(std::true_type{});
        if constexpr (TAIL) {
            // Y(16 rb + 4 v + s, 16 NF + i) for i < 4: in lane 16 s + 4 v + i of
            // the tail, in register v of lane i + 16 s in the 16 x 16 layout
#pragma unroll
            for (int rb = 0; rb < RBN; ++rb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const double y = __shfl(acct[rb], (lane & 48) + 4 * v + (lane & 3), 64);
                    acc[rb][NF][v] = (lane & 15) < 4 ? y : 0.0;
                }
        }
        // scale the rows: D(i, j) of a 16 x 16 block sits in register i / 4 of
        // lane j + 16 (i mod 4)
#pragma unroll
        for (int rb = 0; rb < RBN; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double sc = __shfl(scale, 16 * rb + 4 * v + lane / 16, 64);
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) acc[rb][cb][v] *= sc;
            }
        // Gram of the tile on the matrix cores (blocks ci <= cj; it is symmetric)
#pragma unroll
        for (int rb = 0; rb < RBN; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int ci = 0; ci < NCB; ++ci)
#pragma unroll
                    for (int cj = ci; cj < NCB; ++cj)
                        gacc[ci][cj] = __builtin_amdgcn_mfma_f64_16x16x4f64(acc[rb][ci][v], acc[rb][cj][v],
                                                                            gacc[ci][cj], 0, 0, 0);
        wave_sync();
#pragma unroll
        for (int rb = 0; rb < RBN; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int rw = 16 * rb + 4 * v + lane / 16;
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) {
                    const int col = 16 * cb + lane % 16;
                    if (col < kq) sm[rw * ldy + col] = acc[rb][cb][v];
                }
            }
        wave_sync();
        {
            double *Yt = Yout + (int64_t)r0 * kq;
            const int n = nr * kq;
            for (int e = lane; e < n; e += 64) {
                const int q = e / kq;
                Yt[e] = sm[q * ldy + (e - q * kq)];
            }
        }
    }
#pragma unroll
    for (int ci = 0; ci < NCB; ++ci)
#pragma unroll
        for (int cj = ci; cj < NCB; ++cj)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int a = 16 * ci + 4 * v + lane / 16, b2 = 16 * cj + lane % 16;
                if (a < kq && b2 < kq) {
                    G[a * kq + b2] = gacc[ci][cj][v];
                    if (cj != ci) G[b2 * kq + a] = gacc[ci][cj][v];   // the mirror block
                }
            }
}

// stack_project: rows are Sigma_(i) V_(i)^T rows of the store (its element
// type) for whole blocks, FP64 Partial-SVD rows (scale 1) for boundary blocks.
constexpr int kStackXcds = 8;
template <int KQM>
__device__ __forceinline__ void stack_project_body(StoreView st, const Piece *__restrict__ pieces,
                                                   const double *__restrict__ Mp,
                                                   const StackChunk *__restrict__ chunks,
                                                   const double *__restrict__ Vk,
                                                   double *__restrict__ Y,
                                                   double *__restrict__ GYpart, int nchunks,
                                                   int xcd)
{
    extern __shared__ __align__(16) double sm[];
    // Work-groups go to the eight XCDs round-robin.  With xcd set, work-group
    // w takes chunk (w mod 8) per + w / 8: the chunks are in the order of
    // their first block, so each XCD works through its own range of blocks
    // and keeps their stack rows in its L2.  Without, chunk w.
    const int per = (nchunks + kStackXcds - 1) / kStackXcds;
    const int pos = xcd ? (int)(blockIdx.x % kStackXcds) * per + (int)(blockIdx.x / kStackXcds)
                        : (int)blockIdx.x;
    if (pos >= nchunks) return;
    const StackChunk ch = chunks[pos];
    const int c = (int)st.c, k = st.k;
    const int vt_type = st.f32 ? kElemF32 : kElemF64;
    const size_t vt_es = st.f32 ? sizeof(float) : sizeof(double);
    auto row = [&](int r) {
        const Piece &pc = pieces[ch.piece0 + r / k];
        const int j = r % k;
        if (pc.t_idx >= 0)
            return RowRef{reinterpret_cast<const char *>(Mp + ((int64_t)pc.t_idx * k + j) * c), kElemF64, 1.0};
        return RowRef{static_cast<const char *>(st.Vt) + (pc.blk * k + j) * c * vt_es, vt_type,
                      st.S[pc.blk * k + j]};
    };
    const RowRef fallback{static_cast<const char *>(st.Vt), vt_type, 0.0};
    // FP64 stores: every stack row is FP64; FP32 stores mix FP32 store rows
    // with FP64 Partial-SVD rows
    if (st.f32)
        tile_project<KQM, kMixed>(row, ch.npieces * k, c, ch.kk, Vk + (int64_t)ch.prob * c * kMaxK,
                                  Y + ch.y_off, GYpart + (int64_t)ch.slot * kSlotK, fallback, sm);
    else
        tile_project<KQM, kElemF64>(row, ch.npieces * k, c, ch.kk, Vk + (int64_t)ch.prob * c * kMaxK,
                                    Y + ch.y_off, GYpart + (int64_t)ch.slot * kSlotK, fallback, sm);
}

// project (storage phase): rows of A of the chunk, scale 1.
template <int KQM, typename TA>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(KQM <= 32 ? 2 : 1)))
void project_kernel(const TA *__restrict__ X, int64_t ld, int c, const Chunk *__restrict__ chunks,
                    const double *__restrict__ Vk, double *__restrict__ Y, double *__restrict__ GYpart)
{
    extern __shared__ __align__(16) double sm[];
    const Chunk ch = chunks[blockIdx.x];
    constexpr int type = sizeof(TA) == 8 ? kElemF64 : (sizeof(TA) == 4 ? kElemF32 : kElemBF16);
    const TA *Xc = X + ch.x_off;
    auto row = [&](int r) {
        return RowRef{reinterpret_cast<const char *>(Xc + (int64_t)r * ld), type, 1.0};
    };
    const RowRef fallback{reinterpret_cast<const char *>(Xc), type, 0.0};
    tile_project<KQM, type>(row, ch.rows, c, ch.kk, Vk + (int64_t)ch.prob * c * kMaxK, Y + ch.y_off,
                            GYpart + (int64_t)ch.slot * kSlotK, fallback, sm);
}

// Up to 32 columns the kernel fits two waves per SIMD in registers; wider
// tiles keep the compiler's choice (more registers, no spills).
template <int KQM>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(KQM <= 32 ? 2 : 1))) void stack_project_kernel(
    StoreView st, const Piece *__restrict__ pieces, const double *__restrict__ Mp,
    const StackChunk *__restrict__ chunks, const double *__restrict__ Vk, double *__restrict__ Y,
    double *__restrict__ GYpart, int nchunks, int xcd)
{
    stack_project_body<KQM>(st, pieces, Mp, chunks, Vk, Y, GYpart, nchunks, xcd);
}

template <int KQM>
__global__ __launch_bounds__(64) void stack_project_wide_kernel(
    StoreView st, const Piece *__restrict__ pieces, const double *__restrict__ Mp,
    const StackChunk *__restrict__ chunks, const double *__restrict__ Vk, double *__restrict__ Y,
    double *__restrict__ GYpart, int nchunks, int xcd)
{
    stack_project_body<KQM>(st, pieces, Mp, chunks, Vk, Y, GYpart, nchunks, xcd);
}

template <typename TU>
__global__ __launch_bounds__(kThreads) void utransform_kernel(const double *Y, TU *U, int k,
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
    const double *Yc = Y + ch.y_off;       // Y and U may be the same array (FP64 store)
    TU *Uc = U + ch.y_off;
    for (int r0 = 0; r0 < ch.rows; r0 += RB) {
        const int nr = min(RB, ch.rows - r0);
        __syncthreads();
        for (int e = tid; e < nr * k; e += kThreads) Us[e] = Yc[(int64_t)r0 * k + e];
        __syncthreads();
        for (int e = tid; e < nr * k; e += kThreads) {
            const int rr = e / k, j = e % k;
            double s = 0.0;
            for (int l = 0; l < k; ++l) s = fma(Us[rr * k + l], Fs[l * k + j], s);
            Uc[(int64_t)r0 * k + e] = (TU)s;
        }
    }
}

}  // namespace

template <int KQM, typename TA>
hipError_t run_project(const TA *X, int64_t ld, int c, const Chunk *chunks, int nchunks, int kk,
                       const double *Vk, double *Y, double *GYpart, hipStream_t stream)
{
    const int w = kk + 1 > kPanel + 1 ? kk + 1 : kPanel + 1;
    const size_t lds = (size_t)(64 * w) * sizeof(double);
    project_kernel<KQM, TA><<<nchunks, 64, lds, stream>>>(X, ld, c, chunks, Vk, Y, GYpart);
    return hipGetLastError();
}

template <typename TA>
hipError_t run_project_t(const TA *X, int64_t ld, int c, const Chunk *chunks, int nchunks, int kk,
                         const double *Vk, double *Y, double *GYpart, hipStream_t stream)
{
    switch (prod_ld(kk)) {
#define ZS_PJ_CASE(KQM) \
    case KQM: return run_project<KQM, TA>(X, ld, c, chunks, nchunks, kk, Vk, Y, GYpart, stream);
        ZS_PJ_CASE(4) ZS_PJ_CASE(8) ZS_PJ_CASE(12) ZS_PJ_CASE(16) ZS_PJ_CASE(20)
        ZS_PJ_CASE(24) ZS_PJ_CASE(28) ZS_PJ_CASE(32) ZS_PJ_CASE(48) ZS_PJ_CASE(64)
#undef ZS_PJ_CASE
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_project(const void *X, int x_type, int64_t ld, int c, const Chunk *chunks,
                          int nchunks, int kk, const double *Vk, double *Y, double *GYpart,
                          hipStream_t stream)
{
    if (nchunks <= 0) return hipSuccess;
    if (kk < 1 || kk > kMaxK) return hipErrorInvalidValue;
    timing_begin("project", stream);
    hipError_t e;
    if (x_type == kElemF32)
        e = run_project_t(static_cast<const float *>(X), ld, c, chunks, nchunks, kk, Vk, Y, GYpart, stream);
    else if (x_type == kElemBF16)
        e = run_project_t(static_cast<const uint16_t *>(X), ld, c, chunks, nchunks, kk, Vk, Y, GYpart,
                          stream);
    else
        e = run_project_t(static_cast<const double *>(X), ld, c, chunks, nchunks, kk, Vk, Y, GYpart,
                          stream);
    timing_end("project", stream);
    return e;
}

template <int KQM>
hipError_t run_stack_project(StoreView st, const Piece *pieces, const double *Mp,
                             const StackChunk *chunks, int nchunks, int kq_max, const double *Vk,
                             double *Y, double *GYpart, hipStream_t stream)
{
    // panel (64 x 17) or Y tile (64 x (kq + 1))
    const int w = kq_max + 1 > kPanel + 1 ? kq_max + 1 : kPanel + 1;
    const size_t lds = (size_t)(64 * w) * sizeof(double);
    char key[64];
    snprintf(key, sizeof key, "kq=%d c=%d n=%d", kq_max, (int)st.c, tune_bucket(nchunks));
    return tuned_launch("stack_order", key, 2, 0, stream, [&](int v) {
        const int xcd = v;
        const unsigned grid = xcd ? (unsigned)(kStackXcds * ((nchunks + kStackXcds - 1) / kStackXcds))
                                  : (unsigned)nchunks;
        if constexpr (KQM <= 32)
            stack_project_kernel<KQM><<<grid, 64, lds, stream>>>(st, pieces, Mp, chunks, Vk, Y, GYpart,
                                                                 nchunks, xcd);
        else
            stack_project_wide_kernel<KQM><<<grid, 64, lds, stream>>>(st, pieces, Mp, chunks, Vk, Y,
                                                                      GYpart, nchunks, xcd);
        return hipGetLastError();
    });
}

hipError_t launch_stack_project(StoreView st, const Piece *pieces, const double *Mp,
                                const StackChunk *chunks, int nchunks, int kq_max,
                                const double *Vk, double *Y, double *GYpart, hipStream_t stream)
{
    if (nchunks <= 0) return hipSuccess;
    if (kq_max < 1 || kq_max > kMaxK) return hipErrorInvalidValue;
    timing_begin("stack_project", stream);
    hipError_t e;
    switch (prod_ld(kq_max)) {
#define ZS_SP_CASE(KQM) \
    case KQM: e = run_stack_project<KQM>(st, pieces, Mp, chunks, nchunks, kq_max, Vk, Y, GYpart, stream); break;
        ZS_SP_CASE(4) ZS_SP_CASE(8) ZS_SP_CASE(12) ZS_SP_CASE(16) ZS_SP_CASE(20)
        ZS_SP_CASE(24) ZS_SP_CASE(28) ZS_SP_CASE(32) ZS_SP_CASE(48) ZS_SP_CASE(64)
#undef ZS_SP_CASE
    default: e = hipErrorInvalidValue;
    }
    timing_end("stack_project", stream);
    return e;
}

hipError_t launch_utransform(const double *Y, void *U, int u_f32, int k, const Chunk *chunks,
                             int nchunks, const double *F, hipStream_t stream)
{
    if (nchunks <= 0) return hipSuccess;
    timing_begin("utransform", stream);
    if (u_f32)
        utransform_kernel<float><<<nchunks, kThreads, 0, stream>>>(Y, static_cast<float *>(U), k,
                                                                    chunks, F);
    else
        utransform_kernel<double><<<nchunks, kThreads, 0, stream>>>(Y, static_cast<double *>(U), k,
                                                                     chunks, F);
    hipError_t e = hipGetLastError();
    timing_end("utransform", stream);
    return e;
}

}  // namespace zs
