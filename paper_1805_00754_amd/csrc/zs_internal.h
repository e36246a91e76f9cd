// Internal declarations shared by the HIP kernels and the host runtime of the
// Zoom-SVD library.  Not part of the public ABI (that is include/zoomsvd.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace zs {

constexpr int kThreads = 256;       // work-group size of every kernel
constexpr int kMaxC = 128;          // largest c handled by the LDS-resident eigen-solver
constexpr int kMaxK = 64;           // largest stored / requested rank
constexpr int kSlotK = kMaxK * kMaxK;  // stride of a k x k slot (G_Y partials, F factors)
constexpr int kMaxSweeps = 40;      // Jacobi sweep cap
constexpr double kRankTolFP64 = 1e-11;  // numerical-rank threshold relative to sigma_1

// A run of rows of a tall-skinny matrix X (Gram, projection kernels).
struct Chunk {
    int64_t x_off;    // element offset of the first row in X
    int64_t y_off;    // element offset of the first row in Y (row length kk)
    int32_t rows;     // rows in this chunk
    int32_t prob;     // problem (block or query) the chunk belongs to
    int32_t slot;     // partial-sum slot written by this chunk
    int32_t kk;       // columns of Y (the rank wanted for the problem)
};

// One eigen / finalisation problem (a block of the store or a query).
struct Prob {
    int32_t slot0;    // first partial-sum slot of this problem
    int32_t nslots;   // number of partial-sum slots
    int32_t kk;       // triplets wanted
    int32_t pad;
    double *v_dst;    // V(a, j) written at v_dst[a * v_rs + j * v_cs]
    int64_t v_rs, v_cs;
    double *s_dst;    // kk singular values
    int32_t *k_dst;   // numerical rank kept
};

// One touched block of one query (a piece of the stitched range).
struct Piece {
    int64_t blk;      // block index i
    int64_t m_row;    // first row of its k stack rows in the batch's stack buffer M
    int64_t y_off;    // element offset of its k rows in the batch's Y buffer (row length kq)
    int64_t c_off;    // element offset of its k x kq coefficient matrix in the C buffer
    int64_t out_off;  // element offset of its first output row in the caller's U
    int64_t ldu;      // leading dimension of the caller's U for this query
    int32_t r0, r1;   // kept rows of the block
    int32_t q;        // query index
    int32_t kq;       // requested rank of the query
    int32_t t_idx;    // slot in the Partial-SVD factor buffer, -1 for a whole block
    int32_t pad;
};

// Device-side view of a store.
struct StoreView {
    const double *U;  // t x k, rows of block i hold U_(i)
    const double *Vt; // nb x k x c, block i holds V_(i)^T
    const double *S;  // nb x k
    int64_t t, c, b;
    int32_t k;
};

// ---------------------------------------------------------------- launches
// All launches are asynchronous on `stream` and return the launch status.
hipError_t launch_gram(const double *X, int64_t ld, int c, const Chunk *chunks, int nchunks,
                       double *Gpart, hipStream_t stream);
hipError_t launch_eig(int c, const Prob *probs, int nprob, const double *Gpart, double *Vk,
                      int *conv_flag, hipStream_t stream);
hipError_t launch_project(const double *X, int64_t ld, int c, const Chunk *chunks, int nchunks,
                          const double *Vk, double *Y, double *GYpart, hipStream_t stream);
hipError_t launch_finalize(int c, const Prob *probs, int nprob, const double *GYpart,
                           const double *Vk, double *F, double rank_tol, int *conv_flag,
                           hipStream_t stream);
hipError_t launch_utransform(double *U, int k, const Chunk *chunks, int nchunks, const double *F,
                             hipStream_t stream);
hipError_t launch_partial(StoreView st, const Piece *pieces, const int32_t *pidx, int npartial,
                          double *M, double *T, double rank_tol, int *conv_flag,
                          hipStream_t stream);
hipError_t launch_gather(StoreView st, const Piece *pieces, int npieces, double *M,
                         hipStream_t stream);
hipError_t launch_coef(int k, const Piece *pieces, int npieces, const double *Y, const double *F,
                       const double *T, double *C, hipStream_t stream);
hipError_t launch_blockprod(StoreView st, const Piece *pieces, int npieces, const double *C,
                            double *U, hipStream_t stream);

// Kernel timing hooks (implemented in the runtime).
void timing_begin(const char *name, hipStream_t stream);
void timing_end(const char *name, hipStream_t stream);

}  // namespace zs
