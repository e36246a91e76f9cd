// Tall-skinny Gram panels: G = X^T X over a run of rows of X, accumulated in
// FP64 whatever the element type of X (double, float or bf16).
//
// Used for the block Gram G_i = A_(i)^T A_(i) of the storage phase and for the
// Gram of each query's stacked matrix M = [Sigma'_S V'_S^T; ...; Sigma'_E V'_E^T]
// (Alg. 2, line 3).  Each work-group owns one chunk of rows and one
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

template <typename TA>
void run_gram(const TA *X, int64_t ld, int c, const Chunk *chunks, int nchunks, double *Gpart,
              hipStream_t stream)
{
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
