// Internal declarations shared by the HIP kernels and the host runtime of the
// Zoom-SVD library.  Not part of the public ABI (that is include/zoomsvd.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "zs_types.h"

namespace zs {

// Loads element i of an array of type T as double (bf16 is the upper half of
// an IEEE single).
__device__ __forceinline__ double load_as_double(const double *p, int64_t i) { return p[i]; }
__device__ __forceinline__ double load_as_double(const float *p, int64_t i) { return (double)p[i]; }
__device__ __forceinline__ double load_as_double(const uint16_t *p, int64_t i)
{
    return (double)__uint_as_float((uint32_t)p[i] << 16);
}

// Jacobi sweep cap of the current device (tests lower it to force ZS_ENOCONV).
hipError_t set_sweep_cap(int cap);

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
    // Two rounds over the candidates, the faster of each candidate's two
    // times kept: the first launch of a shape also pays for first touches of
    // its buffers, which would count against whichever variant ran first.
    // Every candidate computes the same outputs, so running them again is
    // harmless.
    float ms[kMaxCand] = {0};
    for (int round = 0; round < 2 && e == hipSuccess; ++round) {
        e = hipEventRecord(ev[0], stream);
        for (int v = 0; v < ncand && e == hipSuccess; ++v) {
            e = run(v);
            if (e == hipSuccess) e = hipEventRecord(ev[v + 1], stream);
        }
        if (e == hipSuccess) e = hipEventSynchronize(ev[ncand]);
        if (e == hipSuccess)
            for (int v = 0; v < ncand; ++v) {
                float t = 0.0f;
                (void)hipEventElapsedTime(&t, ev[v], ev[v + 1]);
                ms[v] = round == 0 ? t : (t < ms[v] ? t : ms[v]);
            }
    }
    int best = dflt;
    if (e == hipSuccess) {
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
