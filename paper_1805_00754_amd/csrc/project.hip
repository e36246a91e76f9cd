// Projection of the data on the first-stage eigenvectors, and the in-place
// U formation of the storage phase.
//
//  * project: for a chunk of rows of a block of A, Y = X V_k (rows x kk,
//    written out) and the partial Gram Y^T Y (kk x kk, one slot per chunk).
//  * stack_project: the same for a query's stacked matrix M, whose rows are
//    read where they live: Sigma_(i) V_(i)^T rows of the store for whole
//    blocks, the Partial-SVD rows for boundary blocks (Alg. 2 line 2).  M is
//    never materialised.  (Its own layout is described at the kernel.)
//  * utransform: U_(i) <- Y_(i) F_(i) in place (F = W Sigma^-1 with the sign
//    rule folded in), giving the block's left singular vectors.
//
// project: rows are staged through LDS with coalesced loads, in panels of up
// to 128 columns; V_k stays in LDS for the whole chunk when c <= 128 and is
// staged panel by panel otherwise.  Thread (rg, j) computes column j of RQ
// consecutive rows with independent accumulators, reading two X values per
// 16-byte LDS load.
#include "zs_internal.h"

namespace zs {
namespace {

constexpr int RQ = 4;        // rows per thread
constexpr int kMaxGroups = 16;
constexpr int kPanelCols = 128;  // columns of X and rows of V_k staged at a time

struct TileGeom {
    int kk, cpad, pw, ldx, groups, rb;
};

__host__ __device__ inline TileGeom tile_geom(int c, int kk)
{
    TileGeom g;
    g.kk = kk;
    g.cpad = (c + 1) & ~1;
    g.pw = g.cpad < kPanelCols ? g.cpad : kPanelCols;
    g.ldx = g.pw + 2;
    g.groups = (kThreads / kk) < kMaxGroups ? (kThreads / kk) : kMaxGroups;
    g.rb = g.groups * RQ;
    return g;
}

__host__ __device__ inline size_t project_lds_bytes(int c, int kk)
{
    const TileGeom g = tile_geom(c, kk);
    return (size_t)(g.pw * kk + g.rb * g.ldx + g.rb * kk) * sizeof(double);
}

// acc[r] += sum_a Xs[rg RQ + r][a] Vs[a][j] over the panel's pw columns.
__device__ __forceinline__ void project_panel(const TileGeom &g, const double *Xs, const double *Vs,
                                              int pw, double *acc)
{
    const int tid = threadIdx.x;
    const int j = tid % g.kk, rg = tid / g.kk;
    if (rg >= g.groups) return;
    const double *x0 = Xs + rg * RQ * g.ldx;
#pragma unroll 4
    for (int a = 0; a < pw; a += 2) {
        const double v0 = Vs[a * g.kk + j];
        const double v1 = Vs[(a + 1) * g.kk + j];
#pragma unroll
        for (int r = 0; r < RQ; ++r) {
            const double2 x = *reinterpret_cast<const double2 *>(x0 + r * g.ldx + a);
            acc[r] = fma(x.x, v0, acc[r]);
            acc[r] = fma(x.y, v1, acc[r]);
        }
    }
}

// Y tile rows rr < nr: Ys[rr][j] and Yg + rr * kk.
__device__ __forceinline__ void store_tile(const TileGeom &g, const double *acc, int nr, double *Ys,
                                           double *Yg)
{
    const int tid = threadIdx.x;
    const int j = tid % g.kk, rg = tid / g.kk;
    if (rg >= g.groups) return;
#pragma unroll
    for (int r = 0; r < RQ; ++r) {
        const int rr = rg * RQ + r;
        if (rr < nr) {
            Ys[rr * g.kk + j] = acc[r];
            Yg[(int64_t)rr * g.kk + j] = acc[r];
        }
    }
}

constexpr int EPT = (kMaxK * kMaxK + kThreads - 1) / kThreads;

// gacc[x] += sum_rr Ys[rr][a] Ys[rr][b] for the entries e = tid + x * 256.
__device__ __forceinline__ void gram_accumulate(const double *Ys, int kk, int nr, double *gacc)
{
    const int tid = threadIdx.x;
#pragma unroll
    for (int x = 0; x < EPT; ++x) {
        const int e = tid + x * kThreads;
        if (e < kk * kk) {
            const int a = e / kk, b = e % kk;
            double s0 = 0.0, s1 = 0.0;
            int rr = 0;
            for (; rr + 1 < nr; rr += 2) {
                s0 = fma(Ys[rr * kk + a], Ys[rr * kk + b], s0);
                s1 = fma(Ys[(rr + 1) * kk + a], Ys[(rr + 1) * kk + b], s1);
            }
            if (rr < nr) s0 = fma(Ys[rr * kk + a], Ys[rr * kk + b], s0);
            gacc[x] += s0 + s1;
        }
    }
}

// Rows [p0, p0 + pw) of V_k (c x kk) into Vs, zero beyond c.
__device__ __forceinline__ void load_vk(const TileGeom &g, int c, int p0, const double *vk, double *Vs)
{
    for (int e = threadIdx.x; e < g.pw * g.kk; e += kThreads) {
        const int a = p0 + e / g.kk;
        Vs[e] = a < c ? vk[(int64_t)p0 * g.kk + e] : 0.0;
    }
}

template <typename TA>
__global__ __launch_bounds__(kThreads) void project_kernel(const TA *__restrict__ X, int64_t ld,
                                                           int c, const Chunk *__restrict__ chunks,
                                                           const double *__restrict__ Vk,
                                                           double *__restrict__ Y,
                                                           double *__restrict__ GYpart)
{
    extern __shared__ __align__(16) double smem[];
    const Chunk ch = chunks[blockIdx.x];
    const TileGeom g = tile_geom(c, ch.kk);
    double *Vs = smem;
    double *Xs = Vs + g.pw * g.kk;
    double *Ys = Xs + g.rb * g.ldx;
    const int tid = threadIdx.x;
    const double *vk = Vk + (int64_t)ch.prob * c * kMaxK;
    const bool one_panel = g.pw == g.cpad;        // c <= kPanelCols: V_k staged once
    if (one_panel) load_vk(g, c, 0, vk, Vs);
    double gacc[EPT];
#pragma unroll
    for (int x = 0; x < EPT; ++x) gacc[x] = 0.0;
    const TA *Xc = X + ch.x_off;
    for (int r0 = 0; r0 < ch.rows; r0 += g.rb) {
        const int nr = min(g.rb, ch.rows - r0);
        double acc[RQ];
#pragma unroll
        for (int r = 0; r < RQ; ++r) acc[r] = 0.0;
        for (int p0 = 0; p0 < g.cpad; p0 += g.pw) {
            __syncthreads();
            if (!one_panel) load_vk(g, c, p0, vk, Vs);
            for (int e = tid; e < g.rb * g.pw; e += kThreads) {
                const int rr = e / g.pw, col = p0 + e % g.pw;
                Xs[rr * g.ldx + e % g.pw] =
                    (rr < nr && col < c) ? load_as_double(Xc, (int64_t)(r0 + rr) * ld + col) : 0.0;
            }
            __syncthreads();
            project_panel(g, Xs, Vs, g.pw, acc);
        }
        store_tile(g, acc, nr, Ys, Y + ch.y_off + (int64_t)r0 * ch.kk);
        __syncthreads();
        gram_accumulate(Ys, ch.kk, nr, gacc);
    }
    double *G = GYpart + (int64_t)ch.slot * kSlotK;
#pragma unroll
    for (int x = 0; x < EPT; ++x) {
        const int e = tid + x * kThreads;
        if (e < ch.kk * ch.kk) G[e] = gacc[x];
    }
}

// Orders the wave's LDS accesses (stack_project work-groups are one wave).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// stack_project: one wave per chunk of pieces, tiles of 64 stack rows.  Row r
// of a tile is s_r x_r with x_r = V_(i)^T row j of the store (s_r = sigma_ij)
// for a whole block, or Partial-SVD row j (s_r = 1).  Lane r loads its own
// row, 16 columns at a time (128 contiguous bytes), into an LDS panel, and the
// tile product X V_k runs on the matrix cores (FP64 MFMA 16x16x4; A fragments
// from the LDS panel, B fragments of V_k loaded per panel), four row blocks
// times ceil(kq / 16) column blocks.  Operand layout: A(i, s) in lane i + 16 s,
// B(s, j) in lane j + 16 s, D(i, j) in register i / 4 of lane j + 16 (i mod 4).
// The scaled tile Y = S X V_k goes out through LDS with coalesced stores.  Its
// Gram Y^T Y is accumulated on the matrix cores straight from the D
// fragments: register v of block (rb, cb) holds Y(16 rb + 4 v + s, 16 cb + i)
// in lane i + 16 s, which is the A layout of (Y^T)(16 cb + i, s) and the B
// layout of Y(s, 16 cb' + j), so each pair of column blocks takes 16 MFMAs
// per tile and no LDS traffic.
constexpr int kPanel = 16;
typedef double v4d __attribute__((ext_vector_type(4)));
typedef const double __attribute__((address_space(1))) gdouble;
typedef const float __attribute__((address_space(1))) gfloat;

template <int KQM>
__device__ __forceinline__ void stack_project_body(StoreView st, const Piece *__restrict__ pieces,
                                                   const double *__restrict__ Mp,
                                                   const StackChunk *__restrict__ chunks,
                                                   const double *__restrict__ Vk,
                                                   double *__restrict__ Y,
                                                   double *__restrict__ GYpart)
{
    extern __shared__ __align__(16) double sm[];
    constexpr int NCB = (KQM + 15) / 16;           // 16-column blocks of Y
    const StackChunk ch = chunks[blockIdx.x];
    const int c = (int)st.c, k = st.k, kq = ch.kk;
    const int lane = threadIdx.x;
    const double *__restrict__ V = Vk + (int64_t)ch.prob * c * kMaxK;   // c x kq, row-major
    const int rows = ch.npieces * k;
    const int ldy = kq + 1;
    v4d gacc[NCB][NCB];
#pragma unroll
    for (int ci = 0; ci < NCB; ++ci)
#pragma unroll
        for (int cj = 0; cj < NCB; ++cj) gacc[ci][cj] = (v4d){0.0, 0.0, 0.0, 0.0};

    for (int r0 = 0; r0 < rows; r0 += 64) {
        const int nr = min(64, rows - r0);
        // the lane's stack row: an FP64 Partial-SVD row, or a store row of the
        // store's element type (xf: float); rows past the tile read row 0 of
        // the store with scale 0
        const char *xp = static_cast<const char *>(st.Vt);
        bool xf = st.f32 != 0;
        double scale = 0.0;
        if (lane < nr) {
            const int r = r0 + lane;
            const Piece &pc = pieces[ch.piece0 + r / k];
            const int j = r % k;
            if (pc.t_idx >= 0) {
                xp = reinterpret_cast<const char *>(Mp + ((int64_t)pc.t_idx * k + j) * c);
                xf = false;
                scale = 1.0;
            } else {
                xp += (pc.blk * k + j) * c * (st.f32 ? sizeof(float) : sizeof(double));
                scale = st.S[pc.blk * k + j];
            }
        }
        const gdouble *xd = reinterpret_cast<const gdouble *>(reinterpret_cast<uintptr_t>(xp));
        const gfloat *xs = reinterpret_cast<const gfloat *>(reinterpret_cast<uintptr_t>(xp));
        v4d acc[4][NCB];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = (v4d){0.0, 0.0, 0.0, 0.0};
        // this lane's row, columns a0 .. a0 + 15 (zero past c), and the B
        // fragments B(s, j) = V_k(a0 + 4 t + s, 16 cb + j), zero outside c x kq
        auto load_panel = [&](int a0, double (&v)[kPanel], double (&bf)[NCB][4]) {
            if (xf) {
#pragma unroll
                for (int i = 0; i < kPanel; ++i) v[i] = a0 + i < c ? (double)xs[a0 + i] : 0.0;
            } else {
#pragma unroll
                for (int i = 0; i < kPanel; ++i) v[i] = a0 + i < c ? xd[a0 + i] : 0.0;
            }
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int vr = a0 + 4 * t + lane / 16, vc = 16 * cb + lane % 16;
                    const double x = V[min(vr, c - 1) * kq + min(vc, kq - 1)];
                    bf[cb][t] = (vr < c && vc < kq) ? x : 0.0;
                }
        };
        // up to 32 columns one panel is in flight ahead of the matrix-core
        // work; wider tiles have no registers to spare for it
        constexpr bool kAhead = KQM <= 32;
        double v[kPanel], bn[NCB][4];
        if (kAhead) load_panel(0, v, bn);
        for (int a0 = 0; a0 < c; a0 += kPanel) {
            if (!kAhead) load_panel(a0, v, bn);
            wave_sync();
#pragma unroll
            for (int i = 0; i < kPanel; ++i) sm[lane * (kPanel + 1) + i] = v[i];
            double bf[NCB][4];
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                for (int t = 0; t < 4; ++t) bf[cb][t] = bn[cb][t];
            if (kAhead && a0 + kPanel < c) load_panel(a0 + kPanel, v, bn);
            wave_sync();
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const double a = sm[(16 * rb + lane % 16) * (kPanel + 1) + 4 * t + lane / 16];
#pragma unroll
                    for (int cb = 0; cb < NCB; ++cb)
                        acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bf[cb][t], acc[rb][cb], 0, 0, 0);
                }
        }
        // scale the rows: D(i, j) of a 16 x 16 block sits in register i / 4 of
        // lane j + 16 (i mod 4)
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double sc = __shfl(scale, 16 * rb + 4 * v + lane / 16, 64);
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) acc[rb][cb][v] *= sc;
            }
        // Gram of the tile on the matrix cores
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v)
#pragma unroll
                for (int ci = 0; ci < NCB; ++ci)
#pragma unroll
                    for (int cj = 0; cj < NCB; ++cj)
                        gacc[ci][cj] = __builtin_amdgcn_mfma_f64_16x16x4f64(acc[rb][ci][v], acc[rb][cj][v],
                                                                            gacc[ci][cj], 0, 0, 0);
        wave_sync();
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = 16 * rb + 4 * v + lane / 16;
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) {
                    const int col = 16 * cb + lane % 16;
                    if (col < kq) sm[row * ldy + col] = acc[rb][cb][v];
                }
            }
        wave_sync();
        {
            double *Yt = Y + ch.y_off + (int64_t)r0 * kq;
            const int n = nr * kq;
            for (int e = lane; e < n; e += 64) {
                const int rr = e / kq;
                Yt[e] = sm[rr * ldy + (e - rr * kq)];
            }
        }
    }
    double *G = GYpart + (int64_t)ch.slot * kSlotK;
#pragma unroll
    for (int ci = 0; ci < NCB; ++ci)
#pragma unroll
        for (int cj = 0; cj < NCB; ++cj)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int a = 16 * ci + 4 * v + lane / 16, b2 = 16 * cj + lane % 16;
                if (a < kq && b2 < kq) G[a * kq + b2] = gacc[ci][cj][v];
            }
}

// Up to 32 columns the kernel fits two waves per SIMD in registers; wider
// tiles keep the compiler's choice (more registers, no spills).
template <int KQM>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void stack_project_kernel(
    StoreView st, const Piece *__restrict__ pieces, const double *__restrict__ Mp,
    const StackChunk *__restrict__ chunks, const double *__restrict__ Vk, double *__restrict__ Y,
    double *__restrict__ GYpart)
{
    stack_project_body<KQM>(st, pieces, Mp, chunks, Vk, Y, GYpart);
}

template <int KQM>
__global__ __launch_bounds__(64) void stack_project_wide_kernel(
    StoreView st, const Piece *__restrict__ pieces, const double *__restrict__ Mp,
    const StackChunk *__restrict__ chunks, const double *__restrict__ Vk, double *__restrict__ Y,
    double *__restrict__ GYpart)
{
    stack_project_body<KQM>(st, pieces, Mp, chunks, Vk, Y, GYpart);
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

template <typename TA>
hipError_t run_project(const TA *X, int64_t ld, int c, const Chunk *chunks, int nchunks, int kk,
                       const double *Vk, double *Y, double *GYpart, hipStream_t stream)
{
    const size_t lds = project_lds_bytes(c, kk);
    static size_t cur = 0;
    hipError_t e = ensure_lds((const void *)project_kernel<TA>, lds, cur);
    if (e != hipSuccess) return e;
    project_kernel<TA><<<nchunks, kThreads, lds, stream>>>(X, ld, c, chunks, Vk, Y, GYpart);
    return hipGetLastError();
}

hipError_t launch_project(const void *X, int x_type, int64_t ld, int c, const Chunk *chunks,
                          int nchunks, int kk, const double *Vk, double *Y, double *GYpart,
                          hipStream_t stream)
{
    if (nchunks <= 0) return hipSuccess;
    timing_begin("project", stream);
    hipError_t e;
    if (x_type == kElemF32)
        e = run_project(static_cast<const float *>(X), ld, c, chunks, nchunks, kk, Vk, Y, GYpart, stream);
    else if (x_type == kElemBF16)
        e = run_project(static_cast<const uint16_t *>(X), ld, c, chunks, nchunks, kk, Vk, Y, GYpart,
                        stream);
    else
        e = run_project(static_cast<const double *>(X), ld, c, chunks, nchunks, kk, Vk, Y, GYpart,
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
    if constexpr (KQM <= 32)
        stack_project_kernel<KQM><<<nchunks, 64, lds, stream>>>(st, pieces, Mp, chunks, Vk, Y, GYpart);
    else
        stack_project_wide_kernel<KQM><<<nchunks, 64, lds, stream>>>(st, pieces, Mp, chunks, Vk, Y, GYpart);
    return hipGetLastError();
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
