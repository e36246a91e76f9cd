/*
 * zoomsvd.h -- C ABI of the MI355X (gfx950) Zoom-SVD library.
 *
 * Zoom-SVD (Jang, Choi, Jung, Kang; arXiv 1805.00754) answers "what is the SVD
 * of the rows [t_s, t_e) of a t x c multivariate time series A?" without
 * keeping A.  The storage phase (Sec. 3.2, Alg. 1, Def. 1-2) compresses every
 * b-row block A_(i) into its rank-k SVD U_(i) Sigma_(i) V_(i)^T.  The query
 * phase (Sec. 3.3, Alg. 2) runs a Partial-SVD of the two boundary blocks
 * (Alg. 3, Eqs. (5)-(6)), an SVD of the vertically stacked Sigma_i V_i^T rows
 * (Eqs. (7)-(8)) and the block-diagonal product diag(U_i) U_r of Eq. (9).
 *
 * Conventions shared by every entry point:
 *   - Row-major storage.  A is t x c, row tau = time tick tau (Def. 1).
 *   - Time ranges are 0-based and half-open: [t_s, t_e), n = t_e - t_s rows.
 *     The paper's inclusive [t_s, t_e] is (t_s, t_e + 1) here.
 *   - Block i holds rows [i*b, min((i+1)*b, t)); the last block may be short.
 *   - Singular values are FP64, descending.  A value <= 1e-11 * sigma_1 (FP64
 *     mode; 1e-5 in the FP32/BF16 modes) is numerically zero: its triplet is
 *     zeroed and it does not count in k_out / k_i.
 *   - Sign rule: every returned pair (u_j, v_j) is flipped so that the entry
 *     of v_j with the largest magnitude is positive.
 *   - Device pointers are HIP device memory; host pointers are ordinary host
 *     memory that is read during the call only.
 *   - Every call enqueues its GPU work on `stream` and returns without waiting
 *     for it, except where noted.  Outputs are valid once the stream has
 *     reached that point.  The store is immutable after zs_store_blocks, so
 *     queries on different streams may run concurrently.  The library keeps
 *     scratch per device and stream; calls on one stream from several host
 *     threads take turns in the library's host part, and calls on different
 *     streams do not wait for each other.
 *   - Calls return a zs_status and never throw or abort.  On error nothing is
 *     written to the outputs; zs_last_error() gives a message for the calling
 *     thread.
 */
#ifndef ZOOMSVD_H
#define ZOOMSVD_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ZS_OK = 0,
    ZS_EINVAL = -1,    /* bad argument: null pointer, b < 1, k < 1, k > c, lda < c, ...   */
    ZS_ERANGE = -2,    /* bad query: t_s < 0, t_e > t, t_s >= t_e, k_q < 1 or k_q > k       */
    ZS_ENOMEM = -3,    /* device allocation failed, or the arrays exceed the device memory  */
    ZS_ENOCONV = -4,   /* a Jacobi eigen-solve hit its sweep cap (reported by zs_sync_status) */
    ZS_EDEVICE = -5,   /* a HIP runtime call failed                                         */
    ZS_EUNSUPPORTED = -6 /* a size the library does not handle (c or k above the limits)  */
} zs_status;

typedef enum { ZS_F64 = 0, ZS_F32 = 1, ZS_BF16 = 2 } zs_dtype;          /* element type of A */
typedef enum { ZS_MODE_FP64 = 0, ZS_MODE_FP32 = 1, ZS_MODE_BF16 = 2 } zs_mode; /* bulk arithmetic */

typedef struct zs_store zs_store;   /* opaque; owns the device-resident U_(i), Sigma_(i), V_(i) */

/* Limits of the library: c <= ZS_MAX_C columns and k <= ZS_MAX_K. */
#define ZS_MAX_C 1024
#define ZS_MAX_K 64

/*
 * zs_store_blocks -- storage phase in batch form (Alg. 1 with the rank-k SVD of
 * each complete block; Def. 1 block partition; Def. 2 sets U, S, V).
 *   A      device pointer, t x c row-major with leading dimension lda >= c,
 *          element type a_type.  Read only.  The caller may free it once the
 *          stream has passed this call (the method discards raw data).
 *   t, c   rows (time ticks) and columns (series); t >= 1, 1 <= c <= ZS_MAX_C.
 *   b      block size >= 1.  k: stored rank, 1 <= k <= min(c, ZS_MAX_K).
 *          Block i keeps k_i = min(k, rows_i, numerical rank) triplets.
 *   a_type ZS_F64, ZS_F32 or ZS_BF16; every mode reads every type and widens
 *          it exactly.
 *   mode   arithmetic of the bulk work and storage of the factors:
 *          ZS_MODE_FP64: everything in FP64; U_(i) and V_(i) stored in FP64,
 *            rank threshold 1e-11.
 *          ZS_MODE_FP32: the block Gram A_(i)^T A_(i) (the O(b c^2) term) on
 *            the FP32 matrix cores, A rounded to FP32; ZS_MODE_BF16: on the
 *            BF16 matrix cores, A rounded to bf16 (bf16 input enters
 *            exactly; FP32 mode also takes bf16 input on the BF16 cores).
 *            Both accumulate in FP32 over runs of 32 (FP32) or 128 (BF16)
 *            rows and add the runs in FP64.  The eigen-solve of the Gram
 *            and one refinement sweep (Y = A_(i) V_k from the input values,
 *            Y^T Y and its Jacobi solve, all FP64) follow in FP64, so sigma
 *            is a Rayleigh-Ritz value of the input.  U_(i), V_(i) stored in
 *            FP32, rank threshold 1e-5; queries return U and V in FP32.
 *            Parity targets against FP64: 1e-5 (FP32), 1e-3 (BF16) relative
 *            on sigma.
 *   out    receives the new store.  The library owns its device memory until
 *          zs_store_free.  The call synchronises `stream` once at the end to
 *          check the per-block Jacobi status; on ZS_ENOCONV the store is still
 *          returned (a block used its last sweep) and *out is set.
 */
zs_status zs_store_blocks(const void *A, int64_t t, int64_t c, int64_t lda, zs_dtype a_type,
                          int64_t b, int32_t k, zs_mode mode, hipStream_t stream, zs_store **out);

/*
 * zs_store_blocks_xi -- zs_store_blocks with the paper's energy threshold
 * (Eq. (1), Sec. 2.1; xi = 0.98 in its experiments).  With 0 < xi < 1 every
 * low-rank approximation of the method keeps the smallest rank whose leading
 * squared singular values reach xi times the sum of all of them:
 *   - block i keeps k_i = min(k, rows_i, numerical rank, xi rank of A_(i));
 *     k is then the cap, and columns past k_i are stored as zeros;
 *   - the store remembers xi, and every query on it (zs_query,
 *     zs_query_batch, zs_query_batch_graph) applies the same rule to the
 *     Partial-SVD of its boundary blocks (Alg. 3) and to the SVD of its
 *     stacked matrix (Alg. 2): k_out = min(k_q, numerical rank, xi rank).
 *   The denominator of Eq. (1) is the matrix's squared Frobenius norm (the
 *   trace of its Gram).  xi = 0 or xi = 1 turns the rule off: the results are
 *   then those of zs_store_blocks.  Other arguments and errors as in
 *   zs_store_blocks, plus ZS_EINVAL for xi outside [0, 1] (or NaN).
 */
zs_status zs_store_blocks_xi(const void *A, int64_t t, int64_t c, int64_t lda, zs_dtype a_type,
                             int64_t b, int32_t k, zs_mode mode, double xi, hipStream_t stream,
                             zs_store **out);

/*
 * zs_store_append -- streaming ingest: appends m rows (time ticks t .. t+m-1)
 * to the store.  Rows first fill the store's last block by the incremental
 * update of Alg. 1 (Eqs. (2)-(3)) taken for those rows at once: the last
 * block's [Sigma V^T; new rows] is decomposed by the storage phase, U' Sigma'
 * V'^T, truncated as any block (k, numerical rank, and xi when the store has
 * one), and the block's U becomes diag(U, I) U'.  The remaining rows form new
 * blocks of b rows, compressed as by zs_store_blocks.  With every block of
 * rank <= k the result equals compressing all rows at once; otherwise the
 * last block carries the truncation of both updates.
 *   R      device pointer, m x c row-major, leading dimension ldr >= c,
 *          element type r_type.  Read during the call only.
 *   The store's arrays are reallocated (its device pointers change): no other
 *   call on the store may overlap this one, and a zs_batch_graph captured on
 *   the store before the append must not be replayed after it.  Queries made
 *   after the call see all t + m rows.  Synchronises `stream`.  On an error
 *   the store is unchanged; ZS_ENOCONV as in zs_store_blocks (the rows are
 *   appended).
 */
zs_status zs_store_append(zs_store *st, const void *R, int64_t m, int64_t ldr, zs_dtype r_type,
                          hipStream_t stream);

/*
 * zs_query -- query phase for one range (Alg. 2 with Alg. 3).
 *   [t_s, t_e)  0 <= t_s < t_e <= t.   k_q: requested rank, 1 <= k_q <= k.
 *   U       device, n x k_q row-major, leading dimension ldu >= k_q (n = t_e - t_s).
 *   S       device, k_q doubles.
 *   V       device, c x k_q row-major, leading dimension ldv >= k_q; column j = v_j.
 *   k_out   device int32: the numerical rank kept (<= k_q).  Columns j >= k_out
 *           of U and V and entries of S are zero.
 *   U and V are double in FP64 mode and float in the FP32 / BF16 modes; S is
 *   always double.  Asynchronous on `stream`.
 */
zs_status zs_query(const zs_store *st, int64_t t_s, int64_t t_e, int32_t k_q, void *U, int64_t ldu,
                   double *S, void *V, int64_t ldv, int32_t *k_out, hipStream_t stream);

/*
 * zs_query_noalloc -- zs_query for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, outputs (bit for bit) and errors as
 * zs_query; the call makes no hipMalloc, hipFree, pinned-host allocation or
 * host-to-device copy.  Its intermediate factors and descriptors live in a
 * fixed device scratch of 64 MiB per GPU (allocated with the library's code
 * object, held until the process ends):
 *   - a query needs about 16 * n_blocks * k * k_q + 8 * (c * 64 + c^2 [c > 128]
 *     + 2 * k * c) bytes of it (n_blocks: blocks the range touches); a query
 *     that needs more returns ZS_ENOMEM before any work is enqueued;
 *   - every call on a GPU uses that GPU's one scratch, so calls that overlap
 *     on one GPU (different streams, host threads, or a graph replay beside
 *     an eager call) race: the caller orders them, e.g. on one stream.
 */
zs_status zs_query_noalloc(const zs_store *st, int64_t t_s, int64_t t_e, int32_t k_q, void *U,
                           int64_t ldu, double *S, void *V, int64_t ldv, int32_t *k_out,
                           hipStream_t stream);

/*
 * zs_query_scratch_bytes -- device scratch (bytes) that the query [t_s, t_e)
 * at rank k_q adds to its stream's workspace in zs_query / zs_query_batch
 * (stacked-matrix projections, coefficient blocks, eigenvector blocks,
 * descriptors): with the outputs, what an admission policy must budget per
 * query.  There is one workspace per device and stream, shared by every
 * store queried on that stream; it grows to the largest batch the stream has
 * run and is kept until zs_release_workspaces.  Returns -1 for a null store or a
 * range or rank that zs_query would reject.
 */
int64_t zs_query_scratch_bytes(const zs_store *st, int64_t t_s, int64_t t_e, int32_t k_q);

/*
 * zs_query_batch -- nq independent queries in one set of launches.
 *   t_s, t_e, k_q   host arrays of nq ranges and ranks (same rules as zs_query).
 *   U, S, V         device base pointers (element types as in zs_query); query q writes
 *                     U + u_off[q]  (n_q x k_q[q], leading dimension k_q[q]),
 *                     S + s_off[q]  (k_q[q] doubles),
 *                     V + v_off[q]  (c x k_q[q], leading dimension k_q[q]),
 *                   offsets in elements, host arrays.
 *   k_out           device, nq int32.
 *   Each query's result does not depend on the other queries in the batch.
 */
zs_status zs_query_batch(const zs_store *st, int32_t nq, const int64_t *t_s, const int64_t *t_e,
                         const int32_t *k_q, void *U, const int64_t *u_off, double *S,
                         const int64_t *s_off, void *V, const int64_t *v_off, int32_t *k_out,
                         hipStream_t stream);

/*
 * zs_window_similarity -- the measure of the paper's case study of finding
 * similar time ranges (Sec. 5): u_1, the first left singular vector of the
 * range (Problem 1 at rank 1, computed by the query phase), of the base
 * range [t_s, t_e) and of each earlier window of the same length,
 * [t_s - w*stride, t_e - w*stride) for w = 1..n_windows, all answered as one
 * batch; then the cosine of each window's u_1 with the base's, row by row
 * within the window.
 *   stride      >= 1 rows; the last window must start at >= 0, else ZS_ERANGE.
 *   sim         device, n_windows doubles: sim[w - 1] = <u_base, u_w> /
 *               (|u_base| |u_w|), 0 when either range has rank 0.  Signs
 *               follow the sign rule of the query outputs.
 *   The windows' factors go to the library's scratch for this stream (n
 *   rows per window), not to the caller.  Asynchronous on `stream`.  Errors as
 *   in zs_query_batch, plus ZS_EINVAL for stride < 1 or n_windows < 1.
 */
zs_status zs_window_similarity(const zs_store *st, int64_t t_s, int64_t t_e, int64_t stride,
                               int32_t n_windows, double *sim, hipStream_t stream);

/*
 * zs_query_batch_graph -- the batched query form captured into a HIP graph
 * for repeated replay of one fixed batch (the same ranges, ranks and output
 * buffers every time), e.g. a dashboard that re-reads a set of windows.
 *   Arguments as in zs_query_batch; `stream` runs one eager pass of the batch
 *   (it also writes the outputs) and is synchronised before the capture.
 *   out   receives the graph.  It owns private scratch (descriptors, pieces,
 *         intermediate factors) sized for this batch and keeps pointers to
 *         `st` and to the output buffers: both must outlive the graph, and
 *         the store must not be freed first.
 *   Replays plan nothing on the host and allocate nothing; their results
 *   are bitwise those of zs_query_batch on the same batch.  Errors as in
 *   zs_query_batch, plus ZS_EDEVICE when capture or instantiation fails
 *   (*out is then NULL).
 */
typedef struct zs_batch_graph zs_batch_graph;
zs_status zs_query_batch_graph(const zs_store *st, int32_t nq, const int64_t *t_s,
                               const int64_t *t_e, const int32_t *k_q, void *U,
                               const int64_t *u_off, double *S, const int64_t *s_off, void *V,
                               const int64_t *v_off, int32_t *k_out, hipStream_t stream,
                               zs_batch_graph **out);

/* zs_batch_graph_launch -- replays the batch on `stream` (asynchronous).
 * Replays on one graph must not overlap (they share the graph's scratch). */
zs_status zs_batch_graph_launch(zs_batch_graph *g, hipStream_t stream);

/* zs_batch_graph_free -- releases the graph and its scratch; NULL is a no-op.
 * Every replay must have completed. */
void zs_batch_graph_free(zs_batch_graph *g);

/*
 * zs_store_graph_create -- the storage phase of one fixed input captured into
 * a HIP graph (Alg. 1 in batch form, as zs_store_blocks), for an input that
 * the caller refreshes in place: e.g. a device window of the series that is
 * rewritten and recompressed over and over.
 *   Arguments as in zs_store_blocks (no energy threshold).  The call builds
 *   the store from A once (eagerly on `stream`, which it synchronises), then
 *   captures the storage phase's launches into a graph.
 *   st      receives the store (queried as any store; freed with
 *           zs_store_free after the graph).
 *   g       receives the graph.  It owns private scratch (partial Grams,
 *           eigenvector blocks, descriptors) and keeps the addresses of A and
 *           of the store's arrays: A must stay allocated at the same address
 *           with the same shape.
 * Errors as in zs_store_blocks, plus ZS_EDEVICE when capture or instantiation
 * fails (both outputs NULL).  ZS_ENOCONV: the eager run hit the sweep cap;
 * both outputs are set.
 */
typedef struct zs_store_graph zs_store_graph;
zs_status zs_store_graph_create(const void *A, int64_t t, int64_t c, int64_t lda, zs_dtype a_type,
                                int64_t b, int32_t k, zs_mode mode, hipStream_t stream,
                                zs_store **st, zs_store_graph **g);

/* zs_store_graph_launch -- re-runs the storage phase from A's current contents
 * into the same store (asynchronous on `stream`): no host planning,
 * allocation or synchronisation.  Its results are bitwise those of
 * zs_store_blocks on the same contents.  Queries on the store and other
 * replays of the graph must not overlap a replay; zs_sync_status reports a
 * replay's ZS_ENOCONV. */
zs_status zs_store_graph_launch(zs_store_graph *g, hipStream_t stream);

/* zs_store_graph_free -- releases the graph and its scratch (synchronises the
 * device first); the store stays.  NULL is a no-op. */
void zs_store_graph_free(zs_store_graph *g);

/* Releases the store's device memory (synchronises the device first); NULL is
 * a no-op. */
void zs_store_free(zs_store *st);

/*
 * zs_release_workspaces -- returns the scratch the library keeps for `stream`
 * on the current device: the storage phase's and the queries' workspaces,
 * which otherwise grow to the largest call the stream has run and stay for
 * the life of the process.  Waits for `stream` first.  For callers that
 * retire a stream, or that need the memory back between phases.  The next
 * call on the stream allocates again; captured graphs keep their own
 * scratch and are not affected.  ZS_OK when nothing was kept; ZS_EDEVICE if
 * the stream cannot be synchronised.
 */
zs_status zs_release_workspaces(hipStream_t stream);

/* Device bytes held by the store: the block factors (8 or 4 bytes per element
 * by mode) and the Gram tree of the
 * blocks (2 n2 c x c FP64 matrices, n2 = smallest power of two >= nb), not the
 * per-stream query scratch. */
int64_t zs_store_bytes(const zs_store *st);

/* Shape of a store: any pointer may be null. */
zs_status zs_store_info(const zs_store *st, int64_t *t, int64_t *c, int64_t *b, int32_t *k,
                        int64_t *nb, int32_t *mode);

/*
 * zs_store_get_block -- copies block i's factors (Def. 2) to device buffers:
 *   U  rows_i x k (ld k), S k doubles, V c x k (ld k, column j = v_j),
 *   k_i device int32.  Element type of U and V as in zs_query.  Asynchronous.
 */
zs_status zs_store_get_block(const zs_store *st, int64_t i, void *U, double *S, void *V,
                             int32_t *k_i, hipStream_t stream);

/*
 * zs_sync_status -- waits for `stream` and reports ZS_ENOCONV if any Jacobi
 * eigen-solve enqueued by this store since the last call hit its sweep cap.
 */
zs_status zs_sync_status(const zs_store *st, hipStream_t stream);

/*
 * Autotuner of launch variants.  Some kernels have launch variants that
 * compute the same bits (tile edge of the reduced-precision block Gram,
 * threads per matrix of the c <= 128 eigen-solver, work order of the block
 * product).  The first call with a new shape times each variant once on the
 * call's own data and keeps the fastest, per process and, when the
 * environment variable ZS_AUTOTUNE_CACHE names a file, in that file (read
 * once, appended on every new choice).  ZS_AUTOTUNE=0 in the environment or
 * zs_autotune(0) turns the timing off (cached choices still apply, else each
 * site's default); graph capture and zs_query_noalloc never time.
 *   zs_autotune_force -- forces `variant` at `site` for every shape
 *       (variant < 0 clears it); sites: "gram_lp_tile" (0: 128-column tiles,
 *       1: 64), "eig_tri_threads" (0: 512 threads, 1: 1024),
 *       "blockprod_order" (0: XCD runs, 1: dispatch order).  For tests.
 *   zs_autotune_table -- the choices so far, one "site|key<TAB>variant<TAB>
 *       times in ms" line each; valid until the calling thread's next call.
 */
void zs_autotune(int on);
zs_status zs_autotune_force(const char *site, int variant);
const char *zs_autotune_table(void);

/*
 * zs_set_sweep_cap -- the sweep cap of every Jacobi solve (Rayleigh-Ritz
 * and Partial-SVD steps) on the current device; 40 by default.  For tests of
 * the ZS_ENOCONV path: with a cap of 1, any solve that needs a second sweep
 * stops there and the store call or zs_sync_status reports ZS_ENOCONV (the
 * results are then not converged).  ZS_EINVAL for cap < 1.
 */
zs_status zs_set_sweep_cap(int cap);

/* Thread-local message describing the last error of the calling thread. */
const char *zs_last_error(void);

/* Library version string. */
const char *zs_version(void);

/*
 * Per-kernel timing (diagnostics).  When enabled, every kernel launch of the
 * library is bracketed by HIP events on its stream; zs_timing_get waits for
 * the recorded events and returns, for kernel `name`, the number of launches
 * and the summed duration in milliseconds since the last reset.
 */
void zs_timing_enable(int on);
void zs_timing_reset(void);
zs_status zs_timing_get(const char *name, int64_t *launches, double *total_ms);

#ifdef __cplusplus
}
#endif
#endif /* ZOOMSVD_H */
