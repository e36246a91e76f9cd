// Tall-skinny Gram panels: G = X^T X over a run of rows of X, accumulated in
// FP64 whatever the element type of X (double, float or bf16).
//
// Used for the block Gram G_i = A_(i)^T A_(i) of the storage phase and for the
// Gram of each query's stacked matrix M = [Sigma'_S V'_S^T; ...; Sigma'_E V'_E^T]
// (the stacked SVD of Alg. 2).  Each work-group owns one chunk of rows and one
// (16*TM) x (16*TM) output tile; rows are staged through LDS in panels of RB
// rows with coalesced loads, every thread accumulates a TM x TM register tile.
// Partial Grams of the chunks of one problem go to separate slots and are
// summed in a fixed order by the consumer, so results do not depend on how
// many other problems share the launch.
#include "zs_internal.h"

namespace zs {
namespace {

template <int TM, typename TA>
__global__ __launch_bounds__(kThreads) void gram_kernel(const TA *__restrict__ X, int64_t ld,
                                                        int c, const Chunk *__restrict__ chunks,
                                                        double *__restrict__ Gpart)
{
    constexpr int TILE = 16 * TM;
    constexpr int RB = 16;
    __shared__ __align__(16) double Xi[RB][TILE];
    __shared__ __align__(16) double Xj[RB][TILE];

    const Chunk ch = chunks[blockIdx.x];
    const int ntile = (c + TILE - 1) / TILE;
    int idx = blockIdx.y, ti = 0;
    while (idx >= ntile - ti) { idx -= ntile - ti; ++ti; }
    const int tj = ti + idx;
    const int ci0 = ti * TILE, cj0 = tj * TILE;
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;

    double acc[TM][TM];
#pragma unroll
    for (int m = 0; m < TM; ++m)
#pragma unroll
        for (int n = 0; n < TM; ++n) acc[m][n] = 0.0;

    const TA *Xc = X + ch.x_off;
    for (int r0 = 0; r0 < ch.rows; r0 += RB) {
        for (int e = threadIdx.x; e < RB * TILE; e += kThreads) {
            const int rr = e / TILE, cc = e % TILE;
            const int row = r0 + rr;
            double vi = 0.0, vj = 0.0;
            if (row < ch.rows) {
                const TA *xr = Xc + (int64_t)row * ld;
                if (ci0 + cc < c) vi = load_as_double(xr, ci0 + cc);
                if (cj0 + cc < c) vj = load_as_double(xr, cj0 + cc);
            }
            Xi[rr][cc] = vi;
            Xj[rr][cc] = vj;
        }
        __syncthreads();
#pragma unroll 4
        for (int rr = 0; rr < RB; ++rr) {
            double a[TM], bb[TM];
#pragma unroll
            for (int m = 0; m < TM; ++m) {
                a[m] = Xi[rr][ty * TM + m];
                bb[m] = Xj[rr][tx * TM + m];
            }
#pragma unroll
            for (int m = 0; m < TM; ++m)
#pragma unroll
                for (int n = 0; n < TM; ++n) acc[m][n] = fma(a[m], bb[n], acc[m][n]);
        }
        __syncthreads();
    }

    double *G = Gpart + (int64_t)ch.slot * c * c;
#pragma unroll
    for (int m = 0; m < TM; ++m) {
        const int i = ci0 + ty * TM + m;
        if (i >= c) continue;
#pragma unroll
        for (int n = 0; n < TM; ++n) {
            const int j = cj0 + tx * TM + n;
            if (j >= c) continue;
            G[(int64_t)i * c + j] = acc[m][n];
            if (ti != tj) G[(int64_t)j * c + i] = acc[m][n];
        }
    }
}

}  // namespace

// Matrix-core form for c <= 128 (at most 8 blocks of 16 columns): one chunk
// per work-group column, G = sum over 4-row steps of F_i^T F_j, where F_b is
// the step's 4 x 16 slice of column block b.  With FP64 MFMA 16x16x4 the A
// operand A(i, s) = X(s, 16 ci + i) and the B operand B(s, j) = X(s, 16 cj + j)
// have the same lane layout (element (s, e) of a slice in lane e + 16 s), so
// one load per column block and step feeds every block product of the step.
// Only blocks ci <= cj are formed (the result is symmetric); wave w owns the
// block columns w and NB - 1 - w, which balances the work: NB + 1 blocks per
// wave for even NB.  D(i, j) sits in register i / 4 of lane j + 16 (i mod 4).
typedef double v4d __attribute__((ext_vector_type(4)));

template <int NBM, typename TA>
__global__ __launch_bounds__(kThreads) void gram_mfma_kernel(const TA *__restrict__ X, int64_t ld,
                                                             int c, const Chunk *__restrict__ chunks,
                                                             double *__restrict__ Gpart)
{
    const Chunk ch = chunks[blockIdx.x];
    const int nb = (c + 15) / 16;
    const int lane = threadIdx.x % 64;
    const int w = (int)blockIdx.y * (kThreads / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    if (2 * w > nb - 1) return;                    // no block column for this wave
    const int ca = w, cb = nb - 1 - w;             // owned block columns (ca <= cb)
    const bool two = cb != ca;
    const TA *Xc = X + ch.x_off;
    const int e = lane % 16, s4 = lane / 16;
    v4d acc_a[NBM], acc_b[NBM];
#pragma unroll
    for (int b = 0; b < NBM; ++b) {
        acc_a[b] = (v4d){0.0, 0.0, 0.0, 0.0};
        acc_b[b] = (v4d){0.0, 0.0, 0.0, 0.0};
    }
    // Steps of 4 rows, ST per half-iteration, in two register sets used in
    // turn: one set's loads are in flight while the other feeds the matrix
    // cores.  Every load is issued (row and column clamped, so no load sits
    // under a branch and no wait drains the other set); rows past the chunk
    // are zeroed by an exact multiply when they are used.
    constexpr int ST = NBM <= 8 ? 2 : 1;
    auto load = [&](int r0, double (&f)[ST][NBM]) {
#pragma unroll
        for (int q = 0; q < ST; ++q) {
            const int64_t r = min(r0 + 4 * q + s4, ch.rows - 1);
#pragma unroll
            for (int b = 0; b < NBM; ++b) f[q][b] = load_as_double(Xc, r * ld + min(16 * b + e, c - 1));
        }
    };
    auto steps = [&](int r0, double (&f)[ST][NBM]) {
#pragma unroll
        for (int q = 0; q < ST; ++q) {
            const double keep = r0 + 4 * q + s4 < ch.rows ? 1.0 : 0.0;
#pragma unroll
            for (int b = 0; b < NBM; ++b) f[q][b] *= keep;
            double fa = f[q][0], fb = f[q][0];
#pragma unroll
            for (int b = 1; b < NBM; ++b) {
                if (b == ca) fa = f[q][b];
                if (b == cb) fb = f[q][b];
            }
#pragma unroll
            for (int b = 0; b < NBM; ++b) {
                if (b <= ca) acc_a[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(f[q][b], fa, acc_a[b], 0, 0, 0);
                if (two && b <= cb)
                    acc_b[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(f[q][b], fb, acc_b[b], 0, 0, 0);
            }
        }
    };
    constexpr int H = 4 * ST;                      // rows per half-iteration
    double f1[ST][NBM], f2[ST][NBM];
    load(0, f1);
    for (int r0 = 0; r0 < ch.rows; r0 += 2 * H) {
        load(r0 + H, f2);                          // past the chunk: clamped, unused
        __builtin_amdgcn_sched_barrier(0);
        steps(r0, f1);
        if (r0 + H >= ch.rows) break;
        load(r0 + 2 * H, f1);
        __builtin_amdgcn_sched_barrier(0);
        steps(r0 + H, f2);
    }
    double *G = Gpart + (int64_t)ch.slot * c * c;
    auto put = [&](int bi, int bj, const v4d &d) {  // block (bi, bj) and its transpose
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = 16 * bi + 4 * v + lane / 16, j = 16 * bj + lane % 16;
            if (i < c && j < c) {
                G[(int64_t)i * c + j] = d[v];
                if (bi != bj) G[(int64_t)j * c + i] = d[v];
            }
        }
    };
#pragma unroll
    for (int b = 0; b < NBM; ++b) {
        if (b <= ca) put(b, ca, acc_a[b]);
        if (two && b <= cb) put(b, cb, acc_b[b]);
    }
}

template <typename TA>
void run_gram(const TA *X, int64_t ld, int c, const Chunk *chunks, int nchunks, double *Gpart,
              hipStream_t stream)
{
    // The matrix-core form for c <= 128.  Wider matrices need 16 block columns
    // of accumulators per wave, which leaves one wave per SIMD and exposes the
    // load latency (measured 3x slower than the register-tiled form at c = 256).
    if (c <= 128) {
        const int nb = (c + 15) / 16;
        const int waves = (nb + 1) / 2;            // two block columns per wave
        dim3 grid(nchunks, (waves + kThreads / 64 - 1) / (kThreads / 64));
        gram_mfma_kernel<8, TA><<<grid, kThreads, 0, stream>>>(X, ld, c, chunks, Gpart);
        return;
    }
    const int tm = c <= 16 ? 1 : c <= 32 ? 2 : c <= 64 ? 4 : 8;
    const int tile = 16 * tm;
    const int ntile = (c + tile - 1) / tile;
    dim3 grid(nchunks, ntile * (ntile + 1) / 2);
    switch (tm) {
    case 1: gram_kernel<1, TA><<<grid, kThreads, 0, stream>>>(X, ld, c, chunks, Gpart); break;
    case 2: gram_kernel<2, TA><<<grid, kThreads, 0, stream>>>(X, ld, c, chunks, Gpart); break;
    case 4: gram_kernel<4, TA><<<grid, kThreads, 0, stream>>>(X, ld, c, chunks, Gpart); break;
    default: gram_kernel<8, TA><<<grid, kThreads, 0, stream>>>(X, ld, c, chunks, Gpart); break;
    }
}

hipError_t launch_gram(const void *X, int x_type, int64_t ld, int c, const Chunk *chunks,
                       int nchunks, double *Gpart, hipStream_t stream)
{
    if (nchunks <= 0) return hipSuccess;
    timing_begin("gram", stream);
    if (x_type == kElemF32)
        run_gram(static_cast<const float *>(X), ld, c, chunks, nchunks, Gpart, stream);
    else if (x_type == kElemBF16)
        run_gram(static_cast<const uint16_t *>(X), ld, c, chunks, nchunks, Gpart, stream);
    else
        run_gram(static_cast<const double *>(X), ld, c, chunks, nchunks, Gpart, stream);
    hipError_t e = hipGetLastError();
    timing_end("gram", stream);
    return e;
}

}  // namespace zs
