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

// Loads element i of an array of type T as double (bf16 is the upper half of
// an IEEE single).
__device__ __forceinline__ double load_as_double(const double *p, int64_t i) { return p[i]; }
__device__ __forceinline__ double load_as_double(const float *p, int64_t i) { return (double)p[i]; }
__device__ __forceinline__ double load_as_double(const uint16_t *p, int64_t i)
{
    return (double)__uint_as_float((uint32_t)p[i] << 16);
}

// Row stride of a piece's coefficient matrix C_i (stored transposed, k_q rows
// of prod_ld(k) values, zero beyond k): k rounded up to a size blockprod is
// compiled for.
__host__ __device__ inline int prod_ld(int k)
{
    if (k <= 32) return (k + 3) & ~3;
    return (k + 15) & ~15;
}

// Whole pieces per projection chunk of a query's stack (stack_project, coef).
constexpr int kQueryChunkPieces = 32;

// Projection chunk j of a query whose pieces start at piece0 and whose Y rows
// start at y0 (slot: the chunk's G_Y partial-sum slot).
__host__ __device__ inline StackChunk make_stack_chunk(int32_t j, int32_t np, int32_t k, int32_t kq,
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

// Device address of this device's scratch (looked up once per device).
hipError_t noalloc_scratch(void **ptr);
hipError_t launch_plan_single(const SinglePlan &p, hipStream_t stream);

// ------------------------------------------------------------- autotuner
// Launch variants of one site compute the same bits; the tuner picks the
// fastest per shape key (tune.cpp).
int tune_bucket(int64_t n);              // n rounded up to a power of two
bool tune_enabled();
void tune_suspend(bool on);              // this thread times nothing while set
bool tune_suspended();
int tune_lookup(const char *site, const char *key);   // -1: not chosen yet
void tune_record(const char *site, const char *key, int choice, const float *ms, int n);
bool stream_capturing(hipStream_t stream);

// Launches variant `run(v)` of a site: the cached choice, else (tuning on and
// the stream not capturing) every variant once, timed with events, keeping
// the fastest; else the default.  Every variant leaves the same outputs, so
// the outputs are valid after the timed runs.
template <class F>
hipError_t tuned_launch(const char *site, const char *key, int ncand, int dflt, hipStream_t stream,
                        F &&run)
{
    const int known = tune_lookup(site, key);
    if (known >= 0 && known < ncand) return run(known);
    if (ncand < 2 || !tune_enabled() || stream_capturing(stream)) return run(dflt);
    constexpr int kMaxCand = 4;
    if (ncand > kMaxCand) ncand = kMaxCand;
    hipEvent_t ev[kMaxCand + 1];
    int made = 0;
    hipError_t e = hipSuccess;
    for (; made <= ncand && e == hipSuccess; ++made) e = hipEventCreate(&ev[made]);
    if (e != hipSuccess) {
        for (int i = 0; i + 1 < made; ++i) (void)hipEventDestroy(ev[i]);
        (void)hipGetLastError();
        return run(dflt);
    }
    float ms[kMaxCand] = {0};
    e = hipEventRecord(ev[0], stream);
    for (int v = 0; v < ncand && e == hipSuccess; ++v) {
        e = run(v);
        if (e == hipSuccess) e = hipEventRecord(ev[v + 1], stream);
    }
    if (e == hipSuccess) e = hipEventSynchronize(ev[ncand]);
    int best = dflt;
    if (e == hipSuccess) {
        for (int v = 0; v < ncand; ++v) (void)hipEventElapsedTime(&ms[v], ev[v], ev[v + 1]);
        best = 0;
        for (int v = 1; v < ncand; ++v)
            if (ms[v] < ms[best]) best = v;
        tune_record(site, key, best, ms, ncand);
    }
    for (int i = 0; i <= ncand; ++i) (void)hipEventDestroy(ev[i]);
    return e;
}

// ---------------------------------------------------------------- launches
// All launches are asynchronous on `stream` and return the launch status.
// Arithmetic of the block Gram: FP64 (FP64 mode, and every Gram of stored
// factors), FP32 or BF16 matrix cores (the reduced modes).
enum GramPrec { kGramF64 = 0, kGramF32 = 1, kGramBF16 = 2 };
hipError_t launch_gram(const void *X, int x_type, int64_t ld, int c, const Chunk *chunks,
                       int nchunks, double *Gpart, hipStream_t stream, int prec = kGramF64);
hipError_t launch_eig_tri(int c, int k, const Prob *probs, int nprob, const double *const *gsrc,
                          const double *const *msrc, double *Vk, hipStream_t stream);
hipError_t launch_project(const void *X, int x_type, int64_t ld, int c, const Chunk *chunks,
                          int nchunks, int kk, const double *Vk, double *Y, double *GYpart,
                          hipStream_t stream);
hipError_t launch_stack_project(StoreView st, const Piece *pieces, const double *Mp,
                                const StackChunk *chunks, int nchunks, int kq_max,
                                const double *Vk, double *Y, double *GYpart, hipStream_t stream);
// Overwrites V_k (no longer needed) with V_k W.
hipError_t launch_finalize(int c, int k, const Prob *probs, int nprob, int kk_max,
                           const double *GYpart, double *Vk, double *F, double rank_tol,
                           const double *const *gsrc, const double *const *msrc, double xi,
                           int *conv_flag, hipStream_t stream);
// U <- Y F per chunk; Y is FP64, U has the store's element type (may alias Y
// in FP64 mode).
hipError_t launch_utransform(const double *Y, void *U, int u_f32, int k, const Chunk *chunks,
                             int nchunks, const double *F, hipStream_t stream);
hipError_t launch_leaf_gram(StoreView st, int64_t nleaves, double *tree, int64_t leaf0,
                            hipStream_t stream);
// rows[i][j][:] = sigma_ij V_(i)^T[j][:] in FP64 for every block.
hipError_t launch_scale_rows(StoreView st, int64_t nb, double *rows, hipStream_t stream);
hipError_t launch_zero(double *p, int64_t n, hipStream_t stream);
// Eigen-solver for 128 < c <= 1024 with the matrix in global scratch.
size_t eig_big_scratch_doubles(int c);
hipError_t launch_eig_big(int c, int k, const Prob *probs, int nprob, const double *const *gsrc,
                          const double *const *msrc, double *scratch, double *Vk, hipStream_t stream);
hipError_t launch_tree_level(int c, double *tree, int64_t node0, int64_t nnodes,
                             hipStream_t stream);
hipError_t launch_partial(StoreView st, const Piece *pieces, const int32_t *pidx, int npartial,
                          double *Mp, double *T, double rank_tol, double xi, int *conv_flag,
                          hipStream_t stream);
hipError_t launch_expand_pieces(StoreView st, const QueryDesc *qd, int nq, int max_np, Piece *pieces,
                                hipStream_t stream);
hipError_t launch_coef(int k, int kq_max, const Piece *pieces, const StackChunk *chunks,
                       int nchunks, const double *Y, const double *F, const double *T, double *C,
                       hipStream_t stream);
// Block-major order of the pieces: perm lists the pieces of block 0, then of
// block 1, ... (boff[i] = first position of block i; bcount is nb counters).
hipError_t launch_order_pieces(const Piece *pieces, int npieces, int64_t nb, const int32_t *boff,
                               int32_t *bcount, int32_t *perm, hipStream_t stream);
// Streaming ingest (append.hip).  P = [sigma_j v_j^T rows of block blk (k);
// m1 rows of R (element type r_type, leading dimension ldr)] in FP64.
hipError_t launch_tail_rows(StoreView st, int64_t blk, const void *R, int r_type, int64_t ldr,
                            int64_t m1, double *P, hipStream_t stream);
// Unew (r_tail + m1 rows x k) = [Uold Up[0:k]; Up[k:k+m1]], all k columns wide.
hipError_t launch_tail_u(const void *Uold, int64_t r_tail, const void *Up, int64_t m1, int k, int f32,
                         void *Unew, hipStream_t stream);
// sim[w - 1] = cosine of u_1 of window w with u_1 of the base (window 0); U
// holds nw + 1 vectors of n elements (float when u_f32).
hipError_t launch_cosine(const void *U, int u_f32, int64_t n, int nw, double *sim,
                         hipStream_t stream);
// contiguous: every query's U has leading dimension k_q (rows back to back)
hipError_t launch_blockprod(StoreView st, const Piece *pieces, const int32_t *perm, int npieces,
                            const double *C, void *U, bool contiguous, hipStream_t stream);

// Raises a kernel's dynamic-LDS limit to `bytes` if it is below (the limit
// only grows; `cur` caches the value set).  Clears the error state on failure.
inline hipError_t ensure_lds(const void *kernel, size_t bytes, size_t &cur)
{
    if (bytes <= cur) return hipSuccess;
    hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return e;
    }
    cur = bytes;
    return hipSuccess;
}

// Kernel timing hooks (implemented in the runtime).
void timing_begin(const char *name, hipStream_t stream);
void timing_end(const char *name, hipStream_t stream);

}  // namespace zs
