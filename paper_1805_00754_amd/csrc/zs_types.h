// Plain descriptor types and size rules of the Zoom-SVD library, shared by
// the HIP kernels, the host runtime and host-only checks (no HIP headers).
#pragma once

#include <stddef.h>
#include <stdint.h>

#if defined(__HIPCC__) || defined(__HIP__)
#define ZS_HD __host__ __device__
#else
#define ZS_HD
#endif

namespace zs {


constexpr int kThreads = 256;       // work-group size of every kernel
constexpr int kMaxC = 128;          // largest c handled by the LDS-resident eigen-solver
constexpr int kMaxK = 64;           // largest stored / requested rank
constexpr int kSlotK = kMaxK * kMaxK;  // stride of a k x k slot (G_Y partials, F factors)
constexpr int kMaxSweeps = 40;      // Jacobi sweep cap
constexpr double kRankTolFP64 = 1e-11;  // numerical-rank threshold relative to sigma_1
constexpr double kRankTolF32 = 1e-5;    // the same for stores kept in FP32

// A run of rows of a tall-skinny matrix X (Gram, projection kernels).
struct Chunk {
    int64_t x_off;    // element offset of the first row in X
    int64_t y_off;    // element offset of the first row in Y (row length kk)
    int32_t rows;     // rows in this chunk
    int32_t prob;     // problem (block or query) the chunk belongs to
    int32_t slot;     // partial-sum slot written by this chunk
    int32_t kk;       // columns of Y (the rank wanted for the problem)
};

// A run of whole pieces of one query's stacked matrix (projection kernel).
struct StackChunk {
    int64_t y_off;    // element offset of the chunk's first stack row in Y (row length kk)
    int32_t piece0;   // first piece of the chunk
    int32_t npieces;  // pieces in the chunk (k stack rows each)
    int32_t prob;     // query
    int32_t slot;     // G_Y partial-sum slot
    int32_t kk;       // k_q of the query
    int32_t pad;
};

// One eigen / finalisation problem (a block of the store or a query).
struct Prob {
    int32_t g0, ng;   // c x c Gram terms: gsrc[g0 .. g0+ng)
    int32_t m0, nm;   // k x c row blocks whose Gram is added: msrc[m0 .. m0+nm)
    int32_t y0, ny;   // G_Y partial-sum slots
    int32_t kk;       // triplets wanted
    int32_t v_f32;    // 1: v_dst holds float
    void *v_dst;      // V(a, j) written at v_dst[a * v_rs + j * v_cs]
    int64_t v_rs, v_cs;
    double *s_dst;    // kk singular values
    int32_t *k_dst;   // numerical rank kept
};

// One touched block of one query (a piece of the stitched range).
struct Piece {
    int64_t blk;      // block index i
    int64_t y_off;    // element offset of its k rows in the batch's Y buffer (row length kq)
    int64_t c_off;    // element offset of its k x kq coefficient matrix in the C buffer
    int64_t out_off;  // element offset of its first output row in the caller's U
    int64_t ldu;      // leading dimension of the caller's U for this query
    int32_t r0, r1;   // kept rows of the block
    int32_t q;        // query index
    int32_t kq;       // requested rank of the query
    int32_t t_idx;    // Partial-SVD slot (stack rows Mp, factor T), -1 for a whole block
    int32_t pad;
};

// One query of a batch, as the piece expansion kernel reads it (the O(1)
// per-query part of the plan; the O(pieces) part is expanded on the device).
struct QueryDesc {
    int64_t S;        // first touched block
    int64_t ts;       // t_s
    int64_t piece0;   // index of the first piece
    int64_t y0, c0;   // element offsets of the first piece in Y and C
    int64_t u_off;    // element offset of the query's U
    int64_t ldu;      // its leading dimension
    int32_t np;       // touched blocks
    int32_t lo, hi;   // first block kept from row lo; last block kept up to row hi
    int32_t kq;
    int32_t t0;       // Partial-SVD slot of the first partial piece
    int32_t first_partial;  // 1 if the first piece goes through the Partial-SVD
};

// Device-side view of a store.  U and Vt hold double in FP64 mode and float
// in the FP32 / BF16 modes (f32 = 1).
struct StoreView {
    const void *U;    // t x k, rows of block i hold U_(i)
    const void *Vt;   // nb x k x c, block i holds V_(i)^T
    const double *S;  // nb x k
    int64_t t, c, b;
    int32_t k;
    int32_t f32;
};

// Element types the storage phase reads A in (zs_dtype order).
enum ElemType { kElemF64 = 0, kElemF32 = 1, kElemBF16 = 2 };

// Row stride of a piece's coefficient matrix C_i (stored transposed, k_q rows
// of prod_ld(k) values, zero beyond k): k rounded up to a size blockprod is
// compiled for.
ZS_HD inline int prod_ld(int k)
{
    if (k <= 32) return (k + 3) & ~3;
    return (k + 15) & ~15;
}

// Whole pieces per projection chunk of a query's stack (stack_project, coef).
constexpr int kQueryChunkPieces = 32;

// Projection chunk j of a query whose pieces start at piece0 and whose Y rows
// start at y0 (slot: the chunk's G_Y partial-sum slot).
ZS_HD inline StackChunk make_stack_chunk(int32_t j, int32_t np, int32_t k, int32_t kq,
                                                      int64_t y0, int64_t piece0, int32_t q,
                                                      int32_t slot)
{
    StackChunk ch;
    const int64_t p = (int64_t)j * kQueryChunkPieces;
    ch.y_off = y0 + p * k * kq;
    ch.piece0 = (int32_t)(piece0 + p);
    ch.npieces = (int32_t)(np - p < kQueryChunkPieces ? np - p : kQueryChunkPieces);
    ch.prob = q;
    ch.slot = slot;
    ch.kk = kq;
    ch.pad = 0;
    return ch;
}

// ------------------------------------------------ no-allocation query scratch
// Size of the fixed device scratch of zs_query_noalloc (one copy per device).
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
// Gram-tree nodes of one query: at most two per level of the tree.
constexpr int kMaxPlanNodes = 96;

// The plan of one query, passed by value to the kernel that writes it into
// the scratch (d_* are the destinations there).
struct SinglePlan {
    QueryDesc qd;
    Prob prob;
    int32_t npidx, ngsrc, nchunks, k;
    int32_t pidx[2];              // pieces that go through the Partial-SVD
    int32_t msrc[2];              // their stack-row slots in Mp
    int64_t gsrc[kMaxPlanNodes];  // Gram-tree nodes of the whole blocks
    int64_t c;
    const double *tree;
    const double *Mp;
    QueryDesc *d_qd;
    Prob *d_prob;
    StackChunk *d_chunks;
    int32_t *d_pidx;
    const double **d_msrc;
    const double **d_gsrc;
    int32_t *d_perm;              // identity order of the pieces
};

}  // namespace zs
