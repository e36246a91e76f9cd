// Projection of the data on the first-stage eigenvectors, and the in-place
// U formation of the storage phase.
//
//  * project: for a chunk of rows of a block of A, Y = X V_k (rows x kk,
//    written out) and the partial Gram Y^T Y (kk x kk, one slot per chunk).
//  * stack_project: the same for a query's stacked matrix M, whose rows are
//    read where they live: Sigma_(i) V_(i)^T rows of the store for whole
//    blocks, the Partial-SVD rows for boundary blocks (Alg. 2 line 2).  M is
//    never materialised.
//  * utransform: U_(i) <- Y_(i) F_(i) in place (F = W Sigma^-1 with the sign
//    rule folded in), giving the block's left singular vectors.
//
// Rows are staged through LDS with coalesced loads; V_k stays in LDS for the
// whole chunk.  Thread (rg, j) computes column j of RQ consecutive rows with
// independent accumulators, reading two X values per 16-byte LDS load.
#include "zs_internal.h"

namespace zs {
namespace {

constexpr int RQ = 4;        // rows per thread
constexpr int kMaxGroups = 16;

struct TileGeom {
    int kk, cpad, ldx, groups, rb;
};

__device__ __forceinline__ TileGeom tile_geom(int c, int kk)
{
    TileGeom g;
    g.kk = kk;
    g.cpad = (c + 1) & ~1;
    g.ldx = g.cpad + 2;
    g.groups = min(kThreads / kk, kMaxGroups);
    g.rb = g.groups * RQ;
    return g;
}

__host__ __device__ inline size_t project_lds_bytes(int c, int kk)
{
    const int cpad = (c + 1) & ~1;
    const int groups = (kThreads / kk) < kMaxGroups ? (kThreads / kk) : kMaxGroups;
    const int rb = groups * RQ;
    return (size_t)(cpad * kk + rb * (cpad + 2) + rb * kk) * sizeof(double);
}

// Y tile: Ys[rr][j] = sum_a Xs[rr][a] Vs[a][j] for rr < nr; also written to
// Yg + rr * kk when Yg is given.
__device__ __forceinline__ void project_tile(const TileGeom &g, const double *Xs, const double *Vs,
                                             int nr, double *Ys, double *Yg)
{
    const int tid = threadIdx.x;
    const int j = tid % g.kk, rg = tid / g.kk;
    if (rg >= g.groups) return;
    double acc[RQ];
#pragma unroll
    for (int r = 0; r < RQ; ++r) acc[r] = 0.0;
    const double *x0 = Xs + rg * RQ * g.ldx;
#pragma unroll 4
    for (int a = 0; a < g.cpad; a += 2) {
        const double v0 = Vs[a * g.kk + j];
        const double v1 = Vs[(a + 1) * g.kk + j];
#pragma unroll
        for (int r = 0; r < RQ; ++r) {
            const double2 x = *reinterpret_cast<const double2 *>(x0 + r * g.ldx + a);
            acc[r] = fma(x.x, v0, acc[r]);
            acc[r] = fma(x.y, v1, acc[r]);
        }
    }
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

__device__ __forceinline__ void load_vk(const TileGeom &g, int c, const double *vk, double *Vs)
{
    for (int e = threadIdx.x; e < g.cpad * g.kk; e += kThreads)
        Vs[e] = (e < c * g.kk) ? vk[e] : 0.0;
}

__global__ __launch_bounds__(kThreads) void project_kernel(const double *__restrict__ X, int64_t ld,
                                                           int c, const Chunk *__restrict__ chunks,
                                                           const double *__restrict__ Vk,
                                                           double *__restrict__ Y,
                                                           double *__restrict__ GYpart)
{
    extern __shared__ __align__(16) double smem[];
    const Chunk ch = chunks[blockIdx.x];
    const TileGeom g = tile_geom(c, ch.kk);
    double *Vs = smem;
    double *Xs = Vs + g.cpad * g.kk;
    double *Ys = Xs + g.rb * g.ldx;
    const int tid = threadIdx.x;
    load_vk(g, c, Vk + (int64_t)ch.prob * c * kMaxK, Vs);
    double gacc[EPT];
#pragma unroll
    for (int x = 0; x < EPT; ++x) gacc[x] = 0.0;
    const double *Xc = X + ch.x_off;
    for (int r0 = 0; r0 < ch.rows; r0 += g.rb) {
        const int nr = min(g.rb, ch.rows - r0);
        __syncthreads();
        for (int e = tid; e < g.rb * g.cpad; e += kThreads) {
            const int rr = e / g.cpad, col = e % g.cpad;
            Xs[rr * g.ldx + col] = (rr < nr && col < c) ? Xc[(int64_t)(r0 + rr) * ld + col] : 0.0;
        }
        __syncthreads();
        project_tile(g, Xs, Vs, nr, Ys, Y + ch.y_off + (int64_t)r0 * ch.kk);
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

__global__ __launch_bounds__(kThreads) void stack_project_kernel(
    StoreView st, const Piece *__restrict__ pieces, const double *__restrict__ Mp,
    const StackChunk *__restrict__ chunks, const double *__restrict__ Vk, double *__restrict__ Y,
    double *__restrict__ GYpart)
{
    extern __shared__ __align__(16) double smem[];
    __shared__ const double *rsrc[kMaxGroups * RQ];
    __shared__ double rscale[kMaxGroups * RQ];
    const StackChunk ch = chunks[blockIdx.x];
    const int c = (int)st.c, k = st.k;
    const TileGeom g = tile_geom(c, ch.kk);
    double *Vs = smem;
    double *Xs = Vs + g.cpad * g.kk;
    double *Ys = Xs + g.rb * g.ldx;
    const int tid = threadIdx.x;
    load_vk(g, c, Vk + (int64_t)ch.prob * c * kMaxK, Vs);
    double gacc[EPT];
#pragma unroll
    for (int x = 0; x < EPT; ++x) gacc[x] = 0.0;
    const int rows = ch.npieces * k;
    for (int r0 = 0; r0 < rows; r0 += g.rb) {
        const int nr = min(g.rb, rows - r0);
        __syncthreads();
        if (tid < nr) {
            const int r = r0 + tid;
            const Piece &pc = pieces[ch.piece0 + r / k];
            const int j = r % k;
            if (pc.t_idx >= 0) {
                rsrc[tid] = Mp + ((int64_t)pc.t_idx * k + j) * c;
                rscale[tid] = 1.0;
            } else {
                rsrc[tid] = st.Vt + (pc.blk * k + j) * c;
                rscale[tid] = st.S[pc.blk * k + j];
            }
        }
        __syncthreads();
        for (int e = tid; e < g.rb * g.cpad; e += kThreads) {
            const int rr = e / g.cpad, col = e % g.cpad;
            Xs[rr * g.ldx + col] = (rr < nr && col < c) ? rsrc[rr][col] * rscale[rr] : 0.0;
        }
        __syncthreads();
        project_tile(g, Xs, Vs, nr, Ys, Y + ch.y_off + (int64_t)r0 * ch.kk);
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
                          int kk, const double *Vk, double *Y, double *GYpart, hipStream_t stream)
{
    if (nchunks <= 0) return hipSuccess;
    const size_t lds = project_lds_bytes(c, kk);
    static size_t cur = 0;
    {
        hipError_t e = ensure_lds((const void *)project_kernel, lds, cur);
        if (e != hipSuccess) return e;
    }
    timing_begin("project", stream);
    project_kernel<<<nchunks, kThreads, lds, stream>>>(X, ld, c, chunks, Vk, Y, GYpart);
    hipError_t e = hipGetLastError();
    timing_end("project", stream);
    return e;
}

hipError_t launch_stack_project(StoreView st, const Piece *pieces, const double *Mp,
                                const StackChunk *chunks, int nchunks, int kq_max,
                                const double *Vk, double *Y, double *GYpart, hipStream_t stream)
{
    if (nchunks <= 0) return hipSuccess;
    // The LDS layout depends on each chunk's kq: size for the worst kq <= kq_max.
    size_t lds = 0;
    for (int kk = 1; kk <= kq_max; ++kk) {
        const size_t b = project_lds_bytes((int)st.c, kk);
        if (b > lds) lds = b;
    }
    static size_t cur = 0;
    {
        hipError_t e = ensure_lds((const void *)stack_project_kernel, lds, cur);
        if (e != hipSuccess) return e;
    }
    timing_begin("stack_project", stream);
    stack_project_kernel<<<nchunks, kThreads, lds, stream>>>(st, pieces, Mp, chunks, Vk, Y, GYpart);
    hipError_t e = hipGetLastError();
    timing_end("stack_project", stream);
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
