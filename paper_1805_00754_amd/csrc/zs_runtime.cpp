// Host runtime of the Zoom-SVD library: the store object, the query planner
// (Alg. 3 index math and the ragged work lists), workspaces, kernel timing and
// the C ABI declared in include/zoomsvd.h.
#include "zoomsvd.h"
#include "zs_internal.h"
#include "plan.h"

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

using namespace zs;

namespace {

thread_local std::string t_err;

zs_status fail(zs_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    return s;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(e_ == hipErrorOutOfMemory ? ZS_ENOMEM : ZS_EDEVICE, "%s: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);                   \
    } while (0)

// ------------------------------------------------------------------ timing
std::mutex g_tmu;
bool g_timing = false;
thread_local bool t_untimed = false;   // launches of this thread are not timed (graph capture)
struct TimedLaunch {
    std::string name;
    hipEvent_t a, b;
};
std::vector<TimedLaunch> g_pending;
std::map<std::string, std::pair<int64_t, double>> g_acc;
thread_local std::map<std::string, hipEvent_t> t_open;

// ------------------------------------------------------------------ buffers
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t need)
    {
        if (need <= bytes) return hipSuccess;
        if (p) {
            hipError_t e = hipFree(p);
            if (e != hipSuccess) return e;
            p = nullptr;
            bytes = 0;
        }
        size_t want = std::max(need, bytes + bytes / 2);
        hipError_t e = hipMalloc(&p, want);
        if (e != hipSuccess) {
            e = hipMalloc(&p, need);
            if (e != hipSuccess) { p = nullptr; return e; }
            want = need;
        }
        bytes = want;
        return hipSuccess;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// Scratch of the query pipeline for one stream (grow-only).
struct Workspace {
    DevBuf Mp, Vk, Y, GY, F, T, C, P, perm, bcount, big, desc;
    DevBuf wU, wS, wV, wK;       // outputs of the windows of zs_window_similarity
    void *host = nullptr;        // pinned staging of the descriptors
    size_t host_bytes = 0;
    hipEvent_t copied = nullptr; // the last upload from `host` has completed
    void release()
    {
        Mp.release(); Vk.release(); Y.release(); GY.release();
        F.release(); T.release(); C.release(); P.release(); perm.release(); bcount.release();
        big.release(); desc.release();
        wU.release(); wS.release(); wV.release(); wK.release();
        if (host) (void)hipHostFree(host);
        if (copied) (void)hipEventDestroy(copied);
        host = nullptr;
        host_bytes = 0;
        copied = nullptr;
    }
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Scratch of the query pipeline, one per (device, stream), grow-only and kept
// until zs_release_workspaces like the storage phase's, so that queries on a
// new store do not allocate again (a batch of the 10^6 x 128 workload on a
// fresh store spent about 0.5 ms in the allocations of its own workspace).
// Calls on one stream are ordered on the device; the lock orders the host
// side of calls made from several threads.  Captured batches keep private
// workspaces.
struct QueryWork {
    std::recursive_mutex mu;
    Workspace w;
};
std::mutex g_qwmu;
std::map<std::pair<int, hipStream_t>, QueryWork *> g_qw;

QueryWork *query_work(int device, hipStream_t stream)
{
    std::lock_guard<std::mutex> lk(g_qwmu);
    QueryWork *&w = g_qw[{device, stream}];
    if (!w) w = new QueryWork();
    return w;
}

// Scratch of the storage phase, one per (device, stream), grow-only and kept
// until zs_release_workspaces, so that repeated stores do not allocate.  A
// store call holds its entry's lock until the stream has synchronised.
struct StoreWork {
    std::mutex mu;
    DevBuf Gpart, Vk, GY, F, Ysc, Big, Rows, desc;
    void *host = nullptr;        // pinned staging of the descriptors
    size_t host_bytes = 0;
    hipEvent_t copied = nullptr; // the last upload from `host` has completed
    void release()
    {
        Gpart.release(); Vk.release(); GY.release(); F.release(); Ysc.release(); Big.release();
        Rows.release(); desc.release();
        if (host) (void)hipHostFree(host);
        if (copied) (void)hipEventDestroy(copied);
        host = nullptr;
        host_bytes = 0;
        copied = nullptr;
    }
};
std::mutex g_swmu;
std::map<std::pair<int, hipStream_t>, StoreWork *> g_sw;

StoreWork *store_work(int device, hipStream_t stream)
{
    std::lock_guard<std::mutex> lk(g_swmu);
    StoreWork *&w = g_sw[{device, stream}];
    if (!w) w = new StoreWork();
    return w;
}

}  // namespace

struct zs_store {
    int64_t t = 0, c = 0, b = 0, nb = 0;
    int32_t k = 0;
    zs_mode mode = ZS_MODE_FP64;
    int device = 0;
    void *base = nullptr;               // one allocation holding the arrays below
    void *U = nullptr, *Vt = nullptr;   // double in FP64 mode, float otherwise
    double *S = nullptr;
    int f32 = 0;                        // U and Vt hold float
    size_t esize() const { return f32 ? sizeof(float) : sizeof(double); }
    // numerical-rank threshold relative to sigma_1: FP32 storage rounds the
    // factors at about 1e-7, so a tighter cut would count rounding as rank
    double rank_tol() const { return f32 ? kRankTolF32 : kRankTolFP64; }
    double xi = 0.0;                    // energy threshold of Eq. (1), 0: none
    int32_t *kvec = nullptr;
    double *tree = nullptr;       // Gram tree: 2 * n2 nodes of c x c (node 0 unused)
    int64_t n2 = 1;               // leaves of the Gram tree (power of two >= nb)
    int *conv = nullptr;          // set by kernels when a Jacobi hits its cap

    StoreView view() const
    {
        StoreView v;
        v.U = U; v.Vt = Vt; v.S = S; v.t = t; v.c = c; v.b = b; v.k = k; v.f32 = f32;
        return v;
    }
    int64_t block_rows(int64_t i) const { return std::min(b, t - i * b); }
};

namespace zs {
void timing_begin(const char *name, hipStream_t stream)
{
    if (!g_timing || t_untimed) return;
    hipEvent_t a;
    if (hipEventCreate(&a) != hipSuccess) return;
    (void)hipEventRecord(a, stream);
    t_open[name] = a;
}

void timing_end(const char *name, hipStream_t stream)
{
    if (!g_timing || t_untimed) return;
    auto it = t_open.find(name);
    if (it == t_open.end()) return;
    hipEvent_t b;
    if (hipEventCreate(&b) != hipSuccess) return;
    (void)hipEventRecord(b, stream);
    std::lock_guard<std::mutex> lk(g_tmu);
    g_pending.push_back({name, it->second, b});
    t_open.erase(it);
}
}  // namespace zs

namespace {

// First-stage eigen-solver: tridiagonalisation with the matrix in registers
// (c <= 128) or in global scratch (c > 128: `big` holds big_doubles(c, nprob)).
size_t big_doubles(int64_t c, int64_t nprob)
{
    return c > kMaxC ? eig_big_scratch_doubles((int)c) * (size_t)nprob : 0;
}

hipError_t first_stage_eig(int c, int k, const Prob *probs, int nprob, const double *const *gsrc,
                           const double *const *msrc, double *Vk, double *big, hipStream_t stream)
{
    if (c > kMaxC) return launch_eig_big(c, k, probs, nprob, gsrc, msrc, big, Vk, stream);
    return launch_eig_tri(c, k, probs, nprob, gsrc, msrc, Vk, stream);
}

// Chunking of tall-skinny row runs for the Gram / projection kernels.
constexpr int kStoreChunkRows = 512;       // Gram chunk rows, c <= 128
constexpr int kStoreChunkRowsWide = 2048;  // c > 128: at least a whole block
constexpr int kProjChunkRows = 256;   // rows per projection wave (storage phase)

// Upload `bytes` of host data to `desc` through a pinned staging buffer
// (grow-only; `copied` marks the end of its last upload, so that it is not
// overwritten while a copy from it may still be in flight).
zs_status upload(DevBuf &desc, void *&host, size_t &host_bytes, hipEvent_t &copied, const void *src,
                 size_t bytes, hipStream_t stream)
{
    if (copied) HIP_TRY(hipEventSynchronize(copied));
    if (bytes > host_bytes) {
        if (host) HIP_TRY(hipHostFree(host));
        host = nullptr;
        size_t want = std::max(bytes, host_bytes * 2);
        HIP_TRY(hipHostMalloc(&host, want, hipHostMallocDefault));
        host_bytes = want;
    }
    if (!copied) HIP_TRY(hipEventCreateWithFlags(&copied, hipEventDisableTiming));
    HIP_TRY(desc.ensure(bytes));
    std::memcpy(host, src, bytes);
    HIP_TRY(hipMemcpyAsync(desc.p, host, bytes, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipEventRecord(copied, stream));
    return ZS_OK;
}

zs_status upload(Workspace &w, const void *src, size_t bytes, hipStream_t stream)
{
    return upload(w.desc, w.host, w.host_bytes, w.copied, src, bytes, stream);
}

// Descriptor blob: several typed arrays packed at 256-byte boundaries.
struct Blob {
    std::vector<char> bytes;
    template <class T> size_t add(const std::vector<T> &v)
    {
        size_t off = align_up(bytes.size(), 256);
        bytes.resize(off + v.size() * sizeof(T) + 1);
        if (!v.empty()) std::memcpy(bytes.data() + off, v.data(), v.size() * sizeof(T));
        return off;
    }
};

// What the launches of a planned batch need besides the workspace: sizes and
// the offsets of the descriptor arrays in the workspace's descriptor buffer.
struct QueryPlan {
    int32_t nq = 0, max_np = 0, kq_max = 1;
    int nchunks = 0, npieces = 0, npartial = 0;
    bool contiguous = true;
    size_t o_chunks = 0, o_probs = 0, o_qds = 0, o_pidx = 0, o_boff = 0, o_gsrc = 0, o_msrc = 0;
    void *U = nullptr;
};

// Plans a batch (Alg. 3 index math, host side), sizes workspace `w` and uploads
// the descriptors to it: through the pinned staging buffer on `stream`, or
// synchronously when `sync_upload` (graphs, whose descriptors must stay put).
zs_status query_plan(zs_store *st, int32_t nq, const int64_t *ts, const int64_t *te,
                     const int32_t *kq, void *U, const int64_t *u_off, const int64_t *ldu,
                     double *S, const int64_t *s_off, void *V, const int64_t *v_off,
                     const int64_t *ldv, int32_t *k_out, hipStream_t stream, Workspace *w,
                     bool sync_upload, QueryPlan &pl)
{
    const int64_t c = st->c;
    const int32_t k = st->k;
    // ---- plan (Alg. 3 index math for every query) ---------------------------------
    // The host computes the O(1) part of each query (plan_one); the pieces
    // themselves are expanded on the device.
    std::vector<QueryDesc> qds(nq);
    VecSink sink;                       // Partial-SVD pieces and slots, tree nodes
    std::vector<StackChunk> chunks;
    std::vector<Prob> probs(nq);
    int64_t y_elems = 0, c_elems = 0, npieces64 = 0;
    int32_t slot = 0, kq_max = 1, max_np = 0;
    const int kp = prod_ld(k);
    for (int32_t q = 0; q < nq; ++q) {
        kq_max = std::max(kq_max, kq[q]);
        const int32_t slot0 = slot;
        plan_one(st, q, ts[q], te[q], kq[q], u_off[q], ldu[q], S + s_off[q],
                 static_cast<char *>(V) + v_off[q] * (int64_t)st->esize(), ldv[q], k_out + q,
                 npieces64, y_elems, c_elems, slot, sink, qds[q], probs[q]);
        const int32_t np = qds[q].np;
        for (int32_t j = 0; j < slot - slot0; ++j)
            chunks.push_back(make_stack_chunk(j, np, k, kq[q], y_elems, npieces64, q, slot0 + j));
        max_np = std::max(max_np, np);
        y_elems += (int64_t)np * k * kq[q];
        c_elems += (int64_t)np * kp * kq[q];
        npieces64 += np;
    }
    // Chunks in the order of their first block (a counting sort, stable): the
    // chunks of different queries that read the same store rows Sigma_(i)
    // V_(i)^T then run together and find them in L2.  Every chunk writes only
    // through its own offsets and slot, so the order changes no result.
    {
        std::vector<int32_t> first(st->nb + 1, 0);
        std::vector<int64_t> key(chunks.size());
        for (size_t i = 0; i < chunks.size(); ++i) {
            const StackChunk &ch = chunks[i];
            key[i] = qds[ch.prob].S + (ch.piece0 - (int64_t)qds[ch.prob].piece0);
            ++first[key[i] + 1];
        }
        for (int64_t b = 0; b < st->nb; ++b) first[b + 1] += first[b];
        std::vector<StackChunk> sorted(chunks.size());
        for (size_t i = 0; i < chunks.size(); ++i) sorted[first[key[i]]++] = chunks[i];
        chunks.swap(sorted);
    }
    std::vector<int32_t> &pidx = sink.pidx;
    std::vector<int64_t> &gsrc_off = sink.gsrc;
    std::vector<int32_t> &msrc_idx = sink.msrc;
    // first position of each block in the block-major order of the pieces
    std::vector<int32_t> boff(st->nb + 1, 0);
    for (int32_t q = 0; q < nq; ++q) {
        boff[qds[q].S] += 1;
        boff[qds[q].S + qds[q].np] -= 1;
    }
    {
        int64_t run = 0, pos = 0;
        for (int64_t i = 0; i < st->nb; ++i) {
            run += boff[i];             // pieces of block i
            boff[i] = (int32_t)pos;
            pos += run;
        }
    }
    if (npieces64 > INT32_MAX)
        return fail(ZS_EUNSUPPORTED, "batch touches %lld blocks (limit %d)", (long long)npieces64,
                    INT32_MAX);
    // ---- workspace ---------------------------------------------------------------
    const int nchunks = (int)chunks.size(), npieces = (int)npieces64;
    const int npartial = (int)pidx.size();
    HIP_TRY(w->Mp.ensure(sizeof(double) * std::max<int64_t>(1, (int64_t)npartial * k * c)));
    HIP_TRY(w->Vk.ensure(sizeof(double) * (size_t)nq * c * kMaxK));
    HIP_TRY(w->Y.ensure(sizeof(double) * std::max<int64_t>(1, y_elems)));
    HIP_TRY(w->GY.ensure(sizeof(double) * (size_t)nchunks * kSlotK));
    HIP_TRY(w->F.ensure(sizeof(double) * (size_t)nq * kSlotK));
    HIP_TRY(w->T.ensure(sizeof(double) * std::max<int64_t>(1, (int64_t)npartial * k * k)));
    HIP_TRY(w->C.ensure(sizeof(double) * std::max<int64_t>(1, c_elems)));
    HIP_TRY(w->P.ensure(sizeof(Piece) * std::max<int64_t>(1, npieces64)));
    HIP_TRY(w->perm.ensure(sizeof(int32_t) * std::max<int64_t>(1, npieces64)));
    HIP_TRY(w->bcount.ensure(sizeof(int32_t) * st->nb));
    double *Mp = w->Mp.as<double>();
    std::vector<const double *> gsrc(gsrc_off.size()), msrc(msrc_idx.size());
    for (size_t i = 0; i < gsrc_off.size(); ++i) gsrc[i] = st->tree + gsrc_off[i] * c * c;
    for (size_t i = 0; i < msrc_idx.size(); ++i) msrc[i] = Mp + (int64_t)msrc_idx[i] * k * c;
    Blob blob;
    const size_t o_chunks = blob.add(chunks), o_probs = blob.add(probs);
    const size_t o_qds = blob.add(qds), o_pidx = blob.add(pidx), o_boff = blob.add(boff);
    const size_t o_gsrc = blob.add(gsrc), o_msrc = blob.add(msrc);
    if (sync_upload) {
        HIP_TRY(w->desc.ensure(blob.bytes.size()));
        HIP_TRY(hipMemcpy(w->desc.p, blob.bytes.data(), blob.bytes.size(), hipMemcpyHostToDevice));
    } else {
        zs_status s = upload(*w, blob.bytes.data(), blob.bytes.size(), stream);
        if (s != ZS_OK) return s;
    }
    pl.nq = nq;
    pl.max_np = max_np;
    pl.kq_max = kq_max;
    pl.nchunks = nchunks;
    pl.npieces = npieces;
    pl.npartial = npartial;
    pl.contiguous = true;
    for (int32_t q = 0; q < nq; ++q) pl.contiguous = pl.contiguous && ldu[q] == kq[q];
    pl.o_chunks = o_chunks;
    pl.o_probs = o_probs;
    pl.o_qds = o_qds;
    pl.o_pidx = o_pidx;
    pl.o_boff = o_boff;
    pl.o_gsrc = o_gsrc;
    pl.o_msrc = o_msrc;
    pl.U = U;
    return ZS_OK;
}

// Device buffers of one planned batch: descriptors and scratch.
struct QueryBufs {
    const StackChunk *chunks;
    const Prob *probs;
    const QueryDesc *qds;
    const int32_t *pidx, *boff;        // boff null: perm is already in place
    const double *const *gsrc;
    const double *const *msrc;
    Piece *P;
    int32_t *perm, *bcount;
    double *Mp, *T, *Vk, *Y, *GY, *F, *C, *big;
};

// Enqueues the kernels of a planned batch on `stream`: no host
// synchronisation and no allocation, so the sequence can be captured into a
// graph.
zs_status query_kernels(zs_store *st, const QueryPlan &pl, const QueryBufs &qb, hipStream_t stream)
{
    const int64_t c = st->c;
    const int32_t k = st->k;
    const StoreView sv = st->view();
    HIP_TRY(launch_expand_pieces(sv, qb.qds, pl.nq, pl.max_np, qb.P, stream));
    HIP_TRY(launch_partial(sv, qb.P, qb.pidx, pl.npartial, qb.Mp, qb.T, st->rank_tol(), st->xi,
                           st->conv, stream));
    HIP_TRY(first_stage_eig((int)c, k, qb.probs, pl.nq, qb.gsrc, qb.msrc, qb.Vk, qb.big, stream));
    HIP_TRY(launch_stack_project(sv, qb.P, qb.Mp, qb.chunks, pl.nchunks, pl.kq_max, qb.Vk, qb.Y,
                                 qb.GY, stream));
    HIP_TRY(launch_finalize((int)c, k, qb.probs, pl.nq, pl.kq_max, qb.GY, qb.Vk, qb.F,
                            st->rank_tol(), qb.gsrc, qb.msrc, st->xi, st->conv, stream));
    HIP_TRY(launch_coef(k, pl.kq_max, qb.P, qb.chunks, pl.nchunks, qb.Y, qb.F, qb.T, qb.C, stream));
    if (qb.boff)
        HIP_TRY(launch_order_pieces(qb.P, pl.npieces, st->nb, qb.boff, qb.bcount, qb.perm, stream));
    HIP_TRY(launch_blockprod(sv, qb.P, qb.perm, pl.npieces, qb.C, pl.U, pl.contiguous, stream));
    return ZS_OK;
}

// The kernels of a batch planned into workspace `w`.
zs_status query_launch(zs_store *st, const QueryPlan &pl, Workspace *w, hipStream_t stream)
{
    HIP_TRY(w->big.ensure(sizeof(double) * std::max<size_t>(1, big_doubles(st->c, pl.nq))));
    char *d = w->desc.as<char>();
    QueryBufs qb;
    qb.chunks = (const StackChunk *)(d + pl.o_chunks);
    qb.probs = (const Prob *)(d + pl.o_probs);
    qb.qds = (const QueryDesc *)(d + pl.o_qds);
    qb.pidx = (const int32_t *)(d + pl.o_pidx);
    qb.boff = (const int32_t *)(d + pl.o_boff);
    qb.gsrc = (const double *const *)(d + pl.o_gsrc);
    qb.msrc = (const double *const *)(d + pl.o_msrc);
    qb.P = w->P.as<Piece>();
    qb.perm = w->perm.as<int32_t>();
    qb.bcount = w->bcount.as<int32_t>();
    qb.Mp = w->Mp.as<double>();
    qb.T = w->T.as<double>();
    qb.Vk = w->Vk.as<double>();
    qb.Y = w->Y.as<double>();
    qb.GY = w->GY.as<double>();
    qb.F = w->F.as<double>();
    qb.C = w->C.as<double>();
    qb.big = w->big.as<double>();
    return query_kernels(st, pl, qb, stream);
}

zs_status query_impl(zs_store *st, int32_t nq, const int64_t *ts, const int64_t *te,
                     const int32_t *kq, void *U, const int64_t *u_off, const int64_t *ldu,
                     double *S, const int64_t *s_off, void *V, const int64_t *v_off,
                     const int64_t *ldv, int32_t *k_out, hipStream_t stream)
{
    QueryWork *qw = query_work(st->device, stream);
    std::lock_guard<std::recursive_mutex> lk(qw->mu);
    Workspace *w = &qw->w;
    QueryPlan pl;
    zs_status s = query_plan(st, nq, ts, te, kq, U, u_off, ldu, S, s_off, V, v_off, ldv, k_out,
                             stream, w, false, pl);
    if (s != ZS_OK) return s;
    return query_launch(st, pl, w, stream);
}

zs_status check_query(const zs_store *st, int64_t ts, int64_t te, int32_t kq)
{
    if (ts < 0 || te > st->t || ts >= te)
        return fail(ZS_ERANGE, "range [%lld, %lld) outside [0, %lld) or empty", (long long)ts,
                    (long long)te, (long long)st->t);
    if (kq < 1 || kq > st->k)
        return fail(ZS_ERANGE, "k_q = %d outside [1, k = %d]", kq, st->k);
    return ZS_OK;
}

// ------------------------------------------------------------ storage phase
// The storage phase is split into its plan (argument checks, allocation, work
// lists, descriptor upload) and its launches (kernels only, no host
// synchronisation and no allocation), so that the launches can be captured
// into a graph (zs_store_graph_create).

zs_status check_store_args(const void *A, int64_t t, int64_t c, int64_t lda, zs_dtype a_type,
                           int64_t b, int32_t k, zs_mode mode, double xi, void *out)
{
    if (!out) return fail(ZS_EINVAL, "out is null");
    if (!(xi >= 0.0 && xi <= 1.0)) return fail(ZS_EINVAL, "xi = %g outside [0, 1]", xi);
    if (!A) return fail(ZS_EINVAL, "A is null");
    if (t < 1) return fail(ZS_EINVAL, "t = %lld < 1", (long long)t);
    if (c < 1) return fail(ZS_EINVAL, "c = %lld < 1", (long long)c);
    if (lda < c) return fail(ZS_EINVAL, "lda = %lld < c = %lld", (long long)lda, (long long)c);
    if (b < 1) return fail(ZS_EINVAL, "b = %lld < 1", (long long)b);
    if (k < 1 || k > c) return fail(ZS_EINVAL, "k = %d outside [1, c = %lld]", k, (long long)c);
    if (c > ZS_MAX_C) return fail(ZS_EUNSUPPORTED, "c = %lld > %d", (long long)c, ZS_MAX_C);
    if (k > ZS_MAX_K) return fail(ZS_EUNSUPPORTED, "k = %d > %d", k, ZS_MAX_K);
    if (a_type != ZS_F64 && a_type != ZS_F32 && a_type != ZS_BF16)
        return fail(ZS_EINVAL, "a_type %d is not a zs_dtype", (int)a_type);
    if (mode != ZS_MODE_FP64 && mode != ZS_MODE_FP32 && mode != ZS_MODE_BF16)
        return fail(ZS_EINVAL, "mode %d is not a zs_mode", (int)mode);
    if (b > (int64_t)1 << 30) return fail(ZS_EINVAL, "b too large");
    return ZS_OK;
}

// A new store with its device arrays (factors, Gram tree, status flag) in one
// allocation; the status flag is cleared on `stream`.
zs_status new_store(int64_t t, int64_t c, int64_t b, int32_t k, zs_mode mode, double xi,
                    hipStream_t stream, zs_store **pst)
{
    zs_store *st = new zs_store();
    st->t = t; st->c = c; st->b = b; st->k = k; st->mode = mode;
    st->xi = xi > 0.0 && xi < 1.0 ? xi : 0.0;
    st->f32 = mode == ZS_MODE_FP64 ? 0 : 1;
    st->nb = (t + b - 1) / b;
    const int64_t nb = st->nb;
    auto bail = [&](zs_status s) {
        zs_store_free(st);
        return s;
    };
    if (hipGetDevice(&st->device) != hipSuccess) return bail(fail(ZS_EDEVICE, "no HIP device"));
    while (st->n2 < nb) st->n2 *= 2;
    const size_t sz[6] = {st->esize() * t * k, st->esize() * nb * k * c, sizeof(double) * nb * k,
                          sizeof(int32_t) * nb, sizeof(double) * 2 * st->n2 * c * c, sizeof(int)};
    size_t off[6], total = 0;
    for (int i = 0; i < 6; ++i) {
        off[i] = total;
        total = align_up(total + sz[i], 256);
    }
    size_t mem_free = 0, mem_total = 0;
    if (hipMemGetInfo(&mem_free, &mem_total) == hipSuccess && total > mem_total)
        return bail(fail(ZS_ENOMEM, "store arrays need %zu bytes; the device has %zu", total,
                         mem_total));
    (void)hipGetLastError();
    hipError_t e = hipMalloc(&st->base, total);
    if (e != hipSuccess)
        return bail(fail(e == hipErrorOutOfMemory ? ZS_ENOMEM : ZS_EDEVICE, "store arrays: %s",
                         hipGetErrorString(e)));
    char *p = static_cast<char *>(st->base);
    st->U = p + off[0];
    st->Vt = p + off[1];
    st->S = reinterpret_cast<double *>(p + off[2]);
    st->kvec = reinterpret_cast<int32_t *>(p + off[3]);
    st->tree = reinterpret_cast<double *>(p + off[4]);
    st->conv = reinterpret_cast<int *>(p + off[5]);
    e = hipMemsetAsync(st->conv, 0, sizeof(int), stream);
    if (e != hipSuccess) return bail(fail(ZS_EDEVICE, "status flag: %s", hipGetErrorString(e)));
    *pst = st;
    return ZS_OK;
}

// What the launches of a planned storage phase need besides the workspace.
struct StorePlan {
    const void *A = nullptr;
    int64_t lda = 0;
    int x_type = kElemF64, gprec = kGramF64;
    int nchunks = 0, npchunks = 0;
    const Chunk *chunks = nullptr, *pchunks = nullptr, *leaf = nullptr;
    const Prob *probs = nullptr;
    const double *const *gsrc = nullptr;
    double *Y = nullptr;
};

// Work lists of the storage phase of `st` from A, scratch sized in `sw`, and
// the descriptors uploaded on `stream` (synchronously when `sync_upload`).
// Work lists: one problem per block.  The Gram works on chunks of at most
// kStoreChunkRows rows (one c x c partial Gram each; one chunk per block for
// c > 128); the projection and the U formation on chunks of kProjChunkRows
// rows (one wave each, one k x k partial G_Y each).
zs_status store_plan(zs_store *st, const void *A, int64_t lda, zs_dtype a_type, StoreWork &sw,
                     hipStream_t stream, bool sync_upload, StorePlan &pl)
{
    const int64_t t = st->t, c = st->c, b = st->b, k = st->k, nb = st->nb;
    std::vector<Chunk> chunks, pchunks;
    std::vector<Prob> probs(nb);
    int32_t slot = 0, pslot = 0;
    for (int64_t i = 0; i < nb; ++i) {
        const int64_t rows = st->block_rows(i);
        Prob pr;
        std::memset(&pr, 0, sizeof pr);
        pr.g0 = slot;
        pr.y0 = pslot;
        const int64_t crows = c > kMaxC ? std::max<int64_t>(kStoreChunkRowsWide, b) : kStoreChunkRows;
        for (int64_t r = 0; r < rows; r += crows) {
            Chunk ch;
            ch.x_off = (i * b + r) * lda;
            ch.y_off = (i * b + r) * k;
            ch.rows = (int32_t)std::min<int64_t>(crows, rows - r);
            ch.prob = (int32_t)i;
            ch.slot = slot++;
            ch.kk = (int32_t)k;
            chunks.push_back(ch);
        }
        for (int64_t r = 0; r < rows; r += kProjChunkRows) {
            Chunk ch;
            ch.x_off = (i * b + r) * lda;
            ch.y_off = (i * b + r) * k;
            ch.rows = (int32_t)std::min<int64_t>(kProjChunkRows, rows - r);
            ch.prob = (int32_t)i;
            ch.slot = pslot++;
            ch.kk = (int32_t)k;
            pchunks.push_back(ch);
        }
        pr.ng = slot - pr.g0;
        pr.ny = pslot - pr.y0;
        pr.kk = (int32_t)k;
        pr.v_dst = static_cast<char *>(st->Vt) + i * k * c * (int64_t)st->esize();  // V_(i)^T
        pr.v_f32 = st->f32;                 // element (a, j) at j * c + a
        pr.v_rs = 1;
        pr.v_cs = c;
        pr.s_dst = st->S + i * k;
        pr.k_dst = st->kvec + i;
        probs[i] = pr;
    }
    pl.nchunks = (int)chunks.size();
    pl.npchunks = (int)pchunks.size();
    HIP_TRY(sw.Gpart.ensure(sizeof(double) * (size_t)pl.nchunks * c * c));
    HIP_TRY(sw.Vk.ensure(sizeof(double) * (size_t)nb * c * kMaxK));
    HIP_TRY(sw.GY.ensure(sizeof(double) * (size_t)pl.npchunks * kSlotK));
    HIP_TRY(sw.F.ensure(sizeof(double) * (size_t)nb * kSlotK));
    // Y = A V_k in FP64: in place in U for an FP64 store, in scratch otherwise
    if (st->f32) HIP_TRY(sw.Ysc.ensure(sizeof(double) * (size_t)t * k));
    pl.Y = st->f32 ? sw.Ysc.as<double>() : static_cast<double *>(st->U);
    HIP_TRY(sw.Big.ensure(sizeof(double) * std::max<size_t>(1, big_doubles(c, nb))));
    if (c > kMaxC) HIP_TRY(sw.Rows.ensure(sizeof(double) * (size_t)nb * k * c));
    std::vector<const double *> gsrc(pl.nchunks);
    for (int s2 = 0; s2 < pl.nchunks; ++s2) gsrc[s2] = sw.Gpart.as<double>() + (int64_t)s2 * c * c;
    std::vector<Chunk> leaf_chunks;           // c > 128: block i's k scaled rows -> leaf i
    if (c > kMaxC) {
        for (int64_t i = 0; i < nb; ++i) {
            Chunk ch;
            ch.x_off = i * k * c;
            ch.y_off = 0;
            ch.rows = (int32_t)k;
            ch.prob = (int32_t)i;
            ch.slot = (int32_t)i;
            ch.kk = (int32_t)k;
            leaf_chunks.push_back(ch);
        }
    }
    Blob blob;
    const size_t o_chunks = blob.add(chunks), o_probs = blob.add(probs), o_gsrc = blob.add(gsrc);
    const size_t o_leaf = blob.add(leaf_chunks), o_pchunks = blob.add(pchunks);
    if (sync_upload) {
        HIP_TRY(sw.desc.ensure(blob.bytes.size()));
        HIP_TRY(hipMemcpy(sw.desc.p, blob.bytes.data(), blob.bytes.size(), hipMemcpyHostToDevice));
    } else {
        zs_status s = upload(sw.desc, sw.host, sw.host_bytes, sw.copied, blob.bytes.data(),
                             blob.bytes.size(), stream);
        if (s != ZS_OK) return s;
    }
    const char *d = sw.desc.as<char>();
    pl.chunks = (const Chunk *)(d + o_chunks);
    pl.probs = (const Prob *)(d + o_probs);
    pl.gsrc = (const double *const *)(d + o_gsrc);
    pl.leaf = (const Chunk *)(d + o_leaf);
    pl.pchunks = (const Chunk *)(d + o_pchunks);
    pl.A = A;
    pl.lda = lda;
    pl.x_type = a_type == ZS_F32 ? kElemF32 : a_type == ZS_BF16 ? kElemBF16 : kElemF64;
    // the bulk Gram in the mode's arithmetic; everything after it in FP64
    pl.gprec = st->mode == ZS_MODE_FP32 ? kGramF32 : st->mode == ZS_MODE_BF16 ? kGramBF16 : kGramF64;
    return ZS_OK;
}

// Enqueues the kernels of a planned storage phase on `stream`.
hipError_t store_kernels(zs_store *st, const StorePlan &pl, StoreWork &sw, hipStream_t stream)
{
    const int64_t c = st->c, k = st->k, nb = st->nb;
#define SK_TRY(expr)                    \
    do {                                \
        hipError_t e_ = (expr);         \
        if (e_ != hipSuccess) return e_; \
    } while (0)
    SK_TRY(launch_gram(pl.A, pl.x_type, pl.lda, (int)c, pl.chunks, pl.nchunks, sw.Gpart.as<double>(),
                       stream, pl.gprec));
    SK_TRY(first_stage_eig((int)c, (int)k, pl.probs, (int)nb, pl.gsrc, nullptr, sw.Vk.as<double>(),
                           sw.Big.as<double>(), stream));
    SK_TRY(launch_project(pl.A, pl.x_type, pl.lda, (int)c, pl.pchunks, pl.npchunks, (int)k,
                          sw.Vk.as<double>(), pl.Y, sw.GY.as<double>(), stream));
    SK_TRY(launch_finalize((int)c, (int)k, pl.probs, (int)nb, (int)k, sw.GY.as<double>(),
                           sw.Vk.as<double>(), sw.F.as<double>(), st->rank_tol(), pl.gsrc, nullptr,
                           st->xi, st->conv, stream));
    SK_TRY(launch_utransform(pl.Y, st->U, st->f32, (int)k, pl.pchunks, pl.npchunks, sw.F.as<double>(),
                             stream));
    // Gram tree over the stored blocks: leaves, then one launch per level.  For
    // c > 128 a leaf is the Gram of the block's rows sigma_ij v_ij^T, formed by
    // the Gram kernel (one chunk of k rows per block); leaves past nb are zero.
    if (c <= kMaxC) {
        SK_TRY(launch_leaf_gram(st->view(), st->n2, st->tree, st->n2, stream));
    } else {
        SK_TRY(launch_scale_rows(st->view(), nb, sw.Rows.as<double>(), stream));
        double *leaves = st->tree + st->n2 * c * c;
        SK_TRY(launch_gram(sw.Rows.as<double>(), kElemF64, c, (int)c, pl.leaf, (int)nb, leaves,
                           stream));
        SK_TRY(launch_zero(leaves + nb * c * c, (st->n2 - nb) * c * c, stream));
    }
    for (int64_t lev = st->n2 / 2; lev >= 1; lev /= 2)
        SK_TRY(launch_tree_level((int)c, st->tree, lev, lev, stream));
#undef SK_TRY
    return hipSuccess;
}

// Reads and clears the store's Jacobi status flag (the stream has synchronised).
zs_status take_conv(zs_store *st, const char *what)
{
    int conv = 0;
    HIP_TRY(hipMemcpy(&conv, st->conv, sizeof(int), hipMemcpyDeviceToHost));
    if (conv) {
        int zero = 0;
        (void)hipMemcpy(st->conv, &zero, sizeof(int), hipMemcpyHostToDevice);
        return fail(ZS_ENOCONV, "%s", what);
    }
    return ZS_OK;
}

}  // namespace

// =============================================================== C ABI
extern "C" {

const char *zs_last_error(void) { return t_err.c_str(); }

const char *zs_version(void) { return "zoomsvd-gfx950 0.1"; }

zs_status zs_store_blocks(const void *A, int64_t t, int64_t c, int64_t lda, zs_dtype a_type,
                          int64_t b, int32_t k, zs_mode mode, hipStream_t stream, zs_store **out)
{
    return zs_store_blocks_xi(A, t, c, lda, a_type, b, k, mode, 0.0, stream, out);
}

zs_status zs_store_blocks_xi(const void *A, int64_t t, int64_t c, int64_t lda, zs_dtype a_type,
                             int64_t b, int32_t k, zs_mode mode, double xi, hipStream_t stream,
                             zs_store **out)
{
    if (out) *out = nullptr;
    zs_status s = check_store_args(A, t, c, lda, a_type, b, k, mode, xi, out);
    if (s != ZS_OK) return s;
    zs_store *st = nullptr;
    s = new_store(t, c, b, k, mode, xi, stream, &st);
    if (s != ZS_OK) return s;
    StoreWork *sw = store_work(st->device, stream);
    std::lock_guard<std::mutex> swlk(sw->mu);
    // the workspace stays allocated; on an error the stream is drained so that
    // no kernel of this call still uses it when the next call reuses it
    auto bail = [&](zs_status e) {
        (void)hipStreamSynchronize(stream);
        zs_store_free(st);
        return e;
    };
    StorePlan pl;
    s = store_plan(st, A, lda, a_type, *sw, stream, false, pl);
    if (s != ZS_OK) return bail(s);
    hipError_t e = store_kernels(st, pl, *sw, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess)
        return bail(fail(e == hipErrorOutOfMemory ? ZS_ENOMEM : ZS_EDEVICE, "storage phase: %s",
                         hipGetErrorString(e)));
    *out = st;
    return take_conv(st, "a block eigen-solve hit the sweep cap");
}

zs_status zs_query(const zs_store *cst, int64_t t_s, int64_t t_e, int32_t k_q, void *U,
                   int64_t ldu, double *S, void *V, int64_t ldv, int32_t *k_out,
                   hipStream_t stream)
{
    if (!cst) return fail(ZS_EINVAL, "store is null");
    zs_status s = check_query(cst, t_s, t_e, k_q);
    if (s != ZS_OK) return s;
    if (!U || !S || !V || !k_out) return fail(ZS_EINVAL, "null output pointer");
    if (ldu < k_q || ldv < k_q) return fail(ZS_EINVAL, "ldu/ldv < k_q");
    zs_store *st = const_cast<zs_store *>(cst);
    const int64_t zero = 0;
    return query_impl(st, 1, &t_s, &t_e, &k_q, U, &zero, &ldu, S, &zero, V, &zero, &ldv, k_out,
                      stream);
}

zs_status zs_query_noalloc(const zs_store *cst, int64_t t_s, int64_t t_e, int32_t k_q, void *U,
                           int64_t ldu, double *S, void *V, int64_t ldv, int32_t *k_out,
                           hipStream_t stream)
{
    if (!cst) return fail(ZS_EINVAL, "store is null");
    zs_status s = check_query(cst, t_s, t_e, k_q);
    if (s != ZS_OK) return s;
    if (!U || !S || !V || !k_out) return fail(ZS_EINVAL, "null output pointer");
    if (ldu < k_q || ldv < k_q) return fail(ZS_EINVAL, "ldu/ldv < k_q");
    zs_store *st = const_cast<zs_store *>(cst);
    const int64_t c = st->c;
    const int32_t k = st->k;
    // the plan, on the host (O(log nb) work), into a by-value descriptor
    SinglePlan p;
    std::memset(&p, 0, sizeof p);
    PlanSink sink{p};
    int32_t nchunks = 0;
    plan_one(st, 0, t_s, t_e, k_q, 0, ldu, S, V, ldv, k_out, 0, 0, 0, nchunks, sink, p.qd, p.prob);
    if (sink.overflow) return fail(ZS_EUNSUPPORTED, "query plan exceeds %d Gram-tree nodes", kMaxPlanNodes);
    const int64_t np = p.qd.np;
    const int64_t npartial = p.npidx;
    // the scratch layout: descriptors, then the intermediate factors
    size_t off = 0;
    auto take = [&](int64_t bytes) {
        const size_t o = off;
        off = align_up(off + (size_t)std::max<int64_t>(bytes, 1), 256);
        return o;
    };
    const size_t o_qd = take(sizeof(QueryDesc)), o_pr = take(sizeof(Prob));
    const size_t o_ch = take((int64_t)sizeof(StackChunk) * nchunks);
    const size_t o_pidx = take(2 * sizeof(int32_t)), o_msrc = take(2 * sizeof(double *));
    const size_t o_gsrc = take((int64_t)sizeof(double *) * p.ngsrc);
    const size_t o_perm = take((int64_t)sizeof(int32_t) * np);
    const size_t o_P = take((int64_t)sizeof(Piece) * np);
    const size_t o_Mp = take(8 * npartial * k * c), o_T = take(8 * npartial * k * k);
    const size_t o_Vk = take(8 * c * kMaxK), o_Y = take(8 * np * k * k_q);
    const size_t o_GY = take(8 * (int64_t)nchunks * kSlotK), o_F = take(8 * (int64_t)kSlotK);
    const size_t o_C = take(8 * np * prod_ld(k) * k_q);
    const size_t o_big = take(8 * (int64_t)big_doubles(c, 1));
    if (off > kNoAllocScratchBytes)
        return fail(ZS_ENOMEM, "query of %lld blocks needs %zu bytes of scratch; the fixed "
                    "no-allocation scratch holds %zu", (long long)np, off, kNoAllocScratchBytes);
    void *vbase = nullptr;
    HIP_TRY(noalloc_scratch(&vbase));
    char *base = static_cast<char *>(vbase);
    p.nchunks = nchunks;
    p.k = k;
    p.c = c;
    p.tree = st->tree;
    p.Mp = reinterpret_cast<const double *>(base + o_Mp);
    p.d_qd = reinterpret_cast<QueryDesc *>(base + o_qd);
    p.d_prob = reinterpret_cast<Prob *>(base + o_pr);
    p.d_chunks = reinterpret_cast<StackChunk *>(base + o_ch);
    p.d_pidx = reinterpret_cast<int32_t *>(base + o_pidx);
    p.d_msrc = reinterpret_cast<const double **>(base + o_msrc);
    p.d_gsrc = reinterpret_cast<const double **>(base + o_gsrc);
    p.d_perm = reinterpret_cast<int32_t *>(base + o_perm);
    QueryPlan pl;
    pl.nq = 1;
    pl.max_np = (int32_t)np;
    pl.kq_max = k_q;
    pl.nchunks = nchunks;
    pl.npieces = (int)np;
    pl.npartial = (int)npartial;
    pl.contiguous = ldu == k_q;
    pl.U = U;
    QueryBufs qb;
    qb.chunks = p.d_chunks;
    qb.probs = p.d_prob;
    qb.qds = p.d_qd;
    qb.pidx = p.d_pidx;
    qb.boff = nullptr;                   // one query: its pieces are in block order
    qb.gsrc = p.d_gsrc;
    qb.msrc = p.d_msrc;
    qb.P = reinterpret_cast<Piece *>(base + o_P);
    qb.perm = p.d_perm;
    qb.bcount = nullptr;
    qb.Mp = reinterpret_cast<double *>(base + o_Mp);
    qb.T = reinterpret_cast<double *>(base + o_T);
    qb.Vk = reinterpret_cast<double *>(base + o_Vk);
    qb.Y = reinterpret_cast<double *>(base + o_Y);
    qb.GY = reinterpret_cast<double *>(base + o_GY);
    qb.F = reinterpret_cast<double *>(base + o_F);
    qb.C = reinterpret_cast<double *>(base + o_C);
    qb.big = reinterpret_cast<double *>(base + o_big);
    // no timing events either: the launches below are all this call makes
    const bool was_untimed = t_untimed, was_suspended = tune_suspended();
    t_untimed = true;
    tune_suspend(true);                  // cached or default launch variants only
    hipError_t e = launch_plan_single(p, stream);
    s = e == hipSuccess ? query_kernels(st, pl, qb, stream)
                        : fail(ZS_EDEVICE, "plan: %s", hipGetErrorString(e));
    t_untimed = was_untimed;
    tune_suspend(was_suspended);
    return s;
}

int64_t zs_query_scratch_bytes(const zs_store *cst, int64_t t_s, int64_t t_e, int32_t k_q)
{
    if (!cst || check_query(cst, t_s, t_e, k_q) != ZS_OK) return -1;
    zs_store *st = const_cast<zs_store *>(cst);
    const int64_t c = st->c, k = st->k;
    SinglePlan p;
    std::memset(&p, 0, sizeof p);
    PlanSink sink{p};
    int32_t nchunks = 0;
    QueryDesc d;
    Prob pr;
    plan_one(st, 0, t_s, t_e, k_q, 0, k_q, nullptr, nullptr, k_q, nullptr, 0, 0, 0, nchunks, sink,
             d, pr);
    const int64_t np = d.np, npartial = p.npidx;
    // the query's share of its stream's workspace (the buffers of query_plan)
    // and of the descriptors
    return 8 * (npartial * k * c + c * kMaxK + np * k * k_q + (int64_t)nchunks * kSlotK + kSlotK +
                npartial * k * k + np * prod_ld((int)k) * k_q + (int64_t)big_doubles(c, 1)) +
           np * (int64_t)(sizeof(Piece) + sizeof(int32_t)) +
           (int64_t)nchunks * sizeof(StackChunk) + (int64_t)(sizeof(Prob) + sizeof(QueryDesc)) +
           8 * (p.ngsrc + 2) + 8;
}

static zs_status check_batch(const zs_store *cst, int32_t nq, const int64_t *t_s, const int64_t *t_e,
                      const int32_t *k_q, void *U, const int64_t *u_off, double *S,
                      const int64_t *s_off, void *V, const int64_t *v_off, int32_t *k_out)
{
    if (!cst) return fail(ZS_EINVAL, "store is null");
    if (nq < 1) return fail(ZS_EINVAL, "nq = %d < 1", nq);
    if (!t_s || !t_e || !k_q || !u_off || !s_off || !v_off)
        return fail(ZS_EINVAL, "null host array");
    if (!U || !S || !V || !k_out) return fail(ZS_EINVAL, "null output pointer");
    for (int32_t q = 0; q < nq; ++q) {
        zs_status s = check_query(cst, t_s[q], t_e[q], k_q[q]);
        if (s != ZS_OK) return s;
        if (u_off[q] < 0 || s_off[q] < 0 || v_off[q] < 0)
            return fail(ZS_EINVAL, "negative output offset for query %d", q);
    }
    return ZS_OK;
}

zs_status zs_query_batch(const zs_store *cst, int32_t nq, const int64_t *t_s, const int64_t *t_e,
                         const int32_t *k_q, void *U, const int64_t *u_off, double *S,
                         const int64_t *s_off, void *V, const int64_t *v_off, int32_t *k_out,
                         hipStream_t stream)
{
    zs_status s = check_batch(cst, nq, t_s, t_e, k_q, U, u_off, S, s_off, V, v_off, k_out);
    if (s != ZS_OK) return s;
    std::vector<int64_t> ld(nq);
    for (int32_t q = 0; q < nq; ++q) ld[q] = k_q[q];
    zs_store *st = const_cast<zs_store *>(cst);
    return query_impl(st, nq, t_s, t_e, k_q, U, u_off, ld.data(), S, s_off, V, v_off, ld.data(),
                      k_out, stream);
}

// The Gram tree of a store from its factors: leaves, then one launch per
// level (leaves past nb are zero).  Synchronises the stream.
static zs_status build_tree(zs_store *st, hipStream_t stream)
{
    const int64_t c = st->c, k = st->k, nb = st->nb;
    if (c <= kMaxC) {
        HIP_TRY(launch_leaf_gram(st->view(), st->n2, st->tree, st->n2, stream));
    } else {
        DevBuf rows, desc;
        std::vector<Chunk> leaf(nb);
        for (int64_t i = 0; i < nb; ++i) {
            std::memset(&leaf[i], 0, sizeof(Chunk));
            leaf[i].x_off = i * k * c;
            leaf[i].rows = (int32_t)k;
            leaf[i].prob = (int32_t)i;
            leaf[i].slot = (int32_t)i;
            leaf[i].kk = (int32_t)k;
        }
        zs_status s = ZS_OK;
        hipError_t e = rows.ensure(sizeof(double) * (size_t)nb * k * c);
        if (e == hipSuccess) e = desc.ensure(sizeof(Chunk) * (size_t)nb);
        if (e == hipSuccess)
            e = hipMemcpy(desc.p, leaf.data(), sizeof(Chunk) * (size_t)nb, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = launch_scale_rows(st->view(), nb, rows.as<double>(), stream);
        double *leaves = st->tree + st->n2 * c * c;
        if (e == hipSuccess)
            e = launch_gram(rows.as<double>(), kElemF64, c, (int)c, desc.as<Chunk>(), (int)nb, leaves,
                            stream);
        if (e == hipSuccess) e = launch_zero(leaves + nb * c * c, (st->n2 - nb) * c * c, stream);
        const hipError_t e2 = hipStreamSynchronize(stream);
        if (e == hipSuccess) e = e2;
        rows.release();
        desc.release();
        if (e != hipSuccess)
            s = fail(e == hipErrorOutOfMemory ? ZS_ENOMEM : ZS_EDEVICE, "Gram tree: %s",
                     hipGetErrorString(e));
        if (s != ZS_OK) return s;
    }
    for (int64_t lev = st->n2 / 2; lev >= 1; lev /= 2)
        HIP_TRY(launch_tree_level((int)c, st->tree, lev, lev, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    return ZS_OK;
}

zs_status zs_store_append(zs_store *st, const void *R, int64_t m, int64_t ldr, zs_dtype r_type,
                          hipStream_t stream)
{
    if (!st) return fail(ZS_EINVAL, "store is null");
    if (!R) return fail(ZS_EINVAL, "R is null");
    if (m < 1) return fail(ZS_EINVAL, "m = %lld < 1", (long long)m);
    if (ldr < st->c) return fail(ZS_EINVAL, "ldr = %lld < c = %lld", (long long)ldr, (long long)st->c);
    if (r_type != ZS_F64 && r_type != ZS_F32 && r_type != ZS_BF16)
        return fail(ZS_EINVAL, "r_type %d is not a zs_dtype", (int)r_type);
    const int64_t t0 = st->t, b = st->b, c = st->c, k = st->k, nb0 = st->nb;
    const int64_t r_tail = t0 - (nb0 - 1) * b;              // rows of the last block
    const int64_t m1 = r_tail < b ? std::min(m, b - r_tail) : 0;   // rows that fill it
    const int64_t m2 = m - m1;                              // rows of new blocks
    const int64_t t1 = t0 + m, nb1 = (t1 + b - 1) / b;
    int64_t n2 = 1;
    while (n2 < nb1) n2 *= 2;
    const int rt = r_type == ZS_F32 ? kElemF32 : r_type == ZS_BF16 ? kElemBF16 : kElemF64;
    const size_t es = st->esize(), rs = r_type == ZS_F64 ? 8 : r_type == ZS_F32 ? 4 : 2;
    zs_store *tp = nullptr, *np = nullptr;
    DevBuf P;
    void *base = nullptr;
    auto cleanup = [&](zs_status s) {
        (void)hipStreamSynchronize(stream);
        if (base) (void)hipFree(base);
        zs_store_free(tp);
        zs_store_free(np);
        P.release();
        return s;
    };
    bool noconv = false;
    // the last block: [Sigma V^T; R[0:m1]] = U' Sigma' V'^T by the storage phase
    if (m1 > 0) {
        hipError_t e = P.ensure(sizeof(double) * (size_t)(k + m1) * c);
        if (e == hipSuccess) e = launch_tail_rows(st->view(), nb0 - 1, R, rt, ldr, m1, P.as<double>(), stream);
        if (e != hipSuccess)
            return cleanup(fail(e == hipErrorOutOfMemory ? ZS_ENOMEM : ZS_EDEVICE, "append: %s",
                                hipGetErrorString(e)));
        zs_status s = zs_store_blocks_xi(P.p, k + m1, c, c, ZS_F64, k + m1, (int32_t)k, st->mode,
                                         st->xi, stream, &tp);
        if (s == ZS_ENOCONV && tp) noconv = true;
        else if (s != ZS_OK) return cleanup(s);
    }
    // whole new blocks from the remaining rows
    if (m2 > 0) {
        zs_status s = zs_store_blocks_xi(static_cast<const char *>(R) + m1 * ldr * (int64_t)rs, m2, c,
                                         ldr, r_type, b, (int32_t)k, st->mode, st->xi, stream, &np);
        if (s == ZS_ENOCONV && np) noconv = true;
        else if (s != ZS_OK) return cleanup(s);
    }
    // the grown arrays, in the layout of zs_store_blocks
    const size_t sz[6] = {es * t1 * k, es * nb1 * k * c, sizeof(double) * nb1 * k,
                          sizeof(int32_t) * nb1, sizeof(double) * 2 * n2 * c * c, sizeof(int)};
    size_t off[6], total = 0;
    for (int i = 0; i < 6; ++i) {
        off[i] = total;
        total = align_up(total + sz[i], 256);
    }
#define AP_TRY(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return cleanup(fail(e_ == hipErrorOutOfMemory ? ZS_ENOMEM : ZS_EDEVICE, "%s: %s", \
                                #expr, hipGetErrorString(e_)));                             \
    } while (0)
    AP_TRY(hipMalloc(&base, total));
    char *p = static_cast<char *>(base);
    char *U1 = p + off[0], *Vt1 = p + off[1];
    double *S1 = reinterpret_cast<double *>(p + off[2]);
    int32_t *K1 = reinterpret_cast<int32_t *>(p + off[3]);
    double *tree1 = reinterpret_cast<double *>(p + off[4]);
    int *conv1 = reinterpret_cast<int *>(p + off[5]);
    const char *U0 = static_cast<const char *>(st->U), *Vt0 = static_cast<const char *>(st->Vt);
    const int64_t bkeep = m1 > 0 ? nb0 - 1 : nb0;          // blocks copied unchanged
    const int64_t rkeep = m1 > 0 ? bkeep * b : t0;          // rows copied unchanged
    const hipMemcpyKind d2d = hipMemcpyDeviceToDevice;
    AP_TRY(hipMemcpyAsync(U1, U0, es * rkeep * k, d2d, stream));
    AP_TRY(hipMemcpyAsync(Vt1, Vt0, es * bkeep * k * c, d2d, stream));
    AP_TRY(hipMemcpyAsync(S1, st->S, sizeof(double) * bkeep * k, d2d, stream));
    AP_TRY(hipMemcpyAsync(K1, st->kvec, sizeof(int32_t) * bkeep, d2d, stream));
    if (m1 > 0) {
        AP_TRY(launch_tail_u(U0 + es * rkeep * k, r_tail, tp->U, m1, (int)k, st->f32, U1 + es * rkeep * k,
                             stream));
        AP_TRY(hipMemcpyAsync(Vt1 + es * bkeep * k * c, tp->Vt, es * k * c, d2d, stream));
        AP_TRY(hipMemcpyAsync(S1 + bkeep * k, tp->S, sizeof(double) * k, d2d, stream));
        AP_TRY(hipMemcpyAsync(K1 + bkeep, tp->kvec, sizeof(int32_t), d2d, stream));
    }
    if (m2 > 0) {
        const int64_t b0 = (t0 + m1) / b;                   // first new block
        AP_TRY(hipMemcpyAsync(U1 + es * (t0 + m1) * k, np->U, es * m2 * k, d2d, stream));
        AP_TRY(hipMemcpyAsync(Vt1 + es * b0 * k * c, np->Vt, es * np->nb * k * c, d2d, stream));
        AP_TRY(hipMemcpyAsync(S1 + b0 * k, np->S, sizeof(double) * np->nb * k, d2d, stream));
        AP_TRY(hipMemcpyAsync(K1 + b0, np->kvec, sizeof(int32_t) * np->nb, d2d, stream));
    }
    AP_TRY(hipMemsetAsync(conv1, 0, sizeof(int), stream));
    AP_TRY(hipStreamSynchronize(stream));
#undef AP_TRY
    // swap in the grown arrays
    void *old = st->base;
    st->base = base;
    base = nullptr;
    st->U = U1;
    st->Vt = Vt1;
    st->S = S1;
    st->kvec = K1;
    st->tree = tree1;
    st->conv = conv1;
    st->t = t1;
    st->nb = nb1;
    st->n2 = n2;
    (void)hipFree(old);
    zs_status s = build_tree(st, stream);
    cleanup(ZS_OK);
    if (s != ZS_OK) return s;
    return noconv ? fail(ZS_ENOCONV, "an appended block's eigen-solve hit the sweep cap") : ZS_OK;
}

zs_status zs_window_similarity(const zs_store *cst, int64_t t_s, int64_t t_e, int64_t stride,
                               int32_t n_windows, double *sim, hipStream_t stream)
{
    if (!cst) return fail(ZS_EINVAL, "store is null");
    if (!sim) return fail(ZS_EINVAL, "sim is null");
    zs_status s = check_query(cst, t_s, t_e, 1);
    if (s != ZS_OK) return s;
    if (stride < 1) return fail(ZS_EINVAL, "stride = %lld < 1", (long long)stride);
    if (n_windows < 1) return fail(ZS_EINVAL, "n_windows = %d < 1", n_windows);
    if (t_s - (int64_t)n_windows * stride < 0)
        return fail(ZS_ERANGE, "window %d would start at %lld < 0", n_windows,
                    (long long)(t_s - (int64_t)n_windows * stride));
    zs_store *st = const_cast<zs_store *>(cst);
    // the base and its earlier windows as one batch of rank-1 queries
    const int32_t nq = n_windows + 1;
    const int64_t n = t_e - t_s;
    std::vector<int64_t> ts(nq), te(nq), u_off(nq), s_off(nq), v_off(nq), ld(nq, 1);
    std::vector<int32_t> kq(nq, 1);
    for (int32_t w = 0; w < nq; ++w) {
        ts[w] = t_s - (int64_t)w * stride;
        te[w] = t_e - (int64_t)w * stride;
        u_off[w] = (int64_t)w * n;
        s_off[w] = w;
        v_off[w] = (int64_t)w * st->c;
    }
    QueryWork *qw = query_work(st->device, stream);
    std::lock_guard<std::recursive_mutex> lk(qw->mu);   // held through the batch below
    Workspace *w = &qw->w;
    HIP_TRY(w->wU.ensure(st->esize() * (size_t)nq * n));
    HIP_TRY(w->wS.ensure(sizeof(double) * (size_t)nq));
    HIP_TRY(w->wV.ensure(st->esize() * (size_t)nq * st->c));
    HIP_TRY(w->wK.ensure(sizeof(int32_t) * (size_t)nq));
    s = query_impl(st, nq, ts.data(), te.data(), kq.data(), w->wU.p, u_off.data(), ld.data(),
                   w->wS.as<double>(), s_off.data(), w->wV.p, v_off.data(), ld.data(),
                   w->wK.as<int32_t>(), stream);
    if (s != ZS_OK) return s;
    HIP_TRY(launch_cosine(w->wU.p, st->f32, n, n_windows, sim, stream));
    return ZS_OK;
}

struct zs_batch_graph {
    zs_store *st = nullptr;
    Workspace *w = nullptr;            // private: the graph's buffers stay put
    QueryPlan pl;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

void zs_batch_graph_free(zs_batch_graph *g)
{
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->w) {
        g->w->release();
        delete g->w;
    }
    delete g;
}

zs_status zs_query_batch_graph(const zs_store *cst, int32_t nq, const int64_t *t_s,
                               const int64_t *t_e, const int32_t *k_q, void *U,
                               const int64_t *u_off, double *S, const int64_t *s_off, void *V,
                               const int64_t *v_off, int32_t *k_out, hipStream_t stream,
                               zs_batch_graph **out)
{
    if (!out) return fail(ZS_EINVAL, "null graph pointer");
    *out = nullptr;
    zs_status s = check_batch(cst, nq, t_s, t_e, k_q, U, u_off, S, s_off, V, v_off, k_out);
    if (s != ZS_OK) return s;
    std::vector<int64_t> ld(nq);
    for (int32_t q = 0; q < nq; ++q) ld[q] = k_q[q];
    zs_batch_graph *g = new zs_batch_graph();
    g->st = const_cast<zs_store *>(cst);
    g->w = new Workspace();
    auto bail = [&](zs_status e) {
        zs_batch_graph_free(g);
        return e;
    };
#define GR_TRY(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return bail(fail(e_ == hipErrorOutOfMemory ? ZS_ENOMEM : ZS_EDEVICE, "%s: %s",    \
                             #expr, hipGetErrorString(e_)));                                \
    } while (0)
    s = query_plan(g->st, nq, t_s, t_e, k_q, U, u_off, ld.data(), S, s_off, V, v_off, ld.data(),
                   k_out, stream, g->w, true, g->pl);
    if (s != ZS_OK) return bail(s);
    // One eager run sizes every lazily grown buffer and sets the kernels' LDS
    // limits, so that the captured launches allocate nothing.
    s = query_launch(g->st, g->pl, g->w, stream);
    if (s != ZS_OK) return bail(s);
    GR_TRY(hipStreamSynchronize(stream));
    hipStream_t cs = nullptr;
    GR_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    t_untimed = true;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        s = query_launch(g->st, g->pl, g->w, cs);
        hipGraph_t graph = nullptr;
        const hipError_t e2 = hipStreamEndCapture(cs, &graph);
        g->graph = graph;
        if (e == hipSuccess) e = e2;
    }
    t_untimed = false;
    (void)hipStreamDestroy(cs);
    if (s != ZS_OK) return bail(s);
    GR_TRY(e);
    GR_TRY(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
#undef GR_TRY
    *out = g;
    return ZS_OK;
}

zs_status zs_batch_graph_launch(zs_batch_graph *g, hipStream_t stream)
{
    if (!g || !g->exec) return fail(ZS_EINVAL, "graph is null");
    HIP_TRY(hipGraphLaunch(g->exec, stream));
    return ZS_OK;
}

struct zs_store_graph {
    zs_store *st = nullptr;
    StoreWork *w = nullptr;            // private: the graph's buffers stay put
    StorePlan pl;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

void zs_store_graph_free(zs_store_graph *g)
{
    if (!g) return;
    (void)hipDeviceSynchronize();
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->w) {
        g->w->Gpart.release(); g->w->Vk.release(); g->w->GY.release(); g->w->F.release();
        g->w->Ysc.release(); g->w->Big.release(); g->w->Rows.release(); g->w->desc.release();
        if (g->w->host) (void)hipHostFree(g->w->host);
        if (g->w->copied) (void)hipEventDestroy(g->w->copied);
        delete g->w;
    }
    delete g;
}

zs_status zs_store_graph_create(const void *A, int64_t t, int64_t c, int64_t lda, zs_dtype a_type,
                                int64_t b, int32_t k, zs_mode mode, hipStream_t stream,
                                zs_store **st_out, zs_store_graph **g_out)
{
    if (st_out) *st_out = nullptr;
    if (g_out) *g_out = nullptr;
    if (!g_out) return fail(ZS_EINVAL, "null graph pointer");
    zs_status s = check_store_args(A, t, c, lda, a_type, b, k, mode, 0.0, st_out);
    if (s != ZS_OK) return s;
    zs_store *st = nullptr;
    s = new_store(t, c, b, k, mode, 0.0, stream, &st);
    if (s != ZS_OK) return s;
    zs_store_graph *g = new zs_store_graph();
    g->st = st;
    g->w = new StoreWork();
    auto bail = [&](zs_status e) {
        (void)hipStreamSynchronize(stream);
        zs_store_graph_free(g);
        zs_store_free(st);
        return e;
    };
#define SG_TRY(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return bail(fail(e_ == hipErrorOutOfMemory ? ZS_ENOMEM : ZS_EDEVICE, "%s: %s",    \
                             #expr, hipGetErrorString(e_)));                                \
    } while (0)
    s = store_plan(st, A, lda, a_type, *g->w, stream, true, g->pl);
    if (s != ZS_OK) return bail(s);
    // One eager run builds the store and sets the kernels' LDS limits, so
    // that the captured launches neither allocate nor configure anything.
    SG_TRY(store_kernels(st, g->pl, *g->w, stream));
    SG_TRY(hipStreamSynchronize(stream));
    const zs_status conv = take_conv(st, "a block eigen-solve hit the sweep cap");
    hipStream_t cs = nullptr;
    SG_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    t_untimed = true;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        e = store_kernels(st, g->pl, *g->w, cs);
        hipGraph_t graph = nullptr;
        const hipError_t e2 = hipStreamEndCapture(cs, &graph);
        g->graph = graph;
        if (e == hipSuccess) e = e2;
    }
    t_untimed = false;
    (void)hipStreamDestroy(cs);
    SG_TRY(e);
    SG_TRY(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
#undef SG_TRY
    *st_out = st;
    *g_out = g;
    return conv;
}

zs_status zs_store_graph_launch(zs_store_graph *g, hipStream_t stream)
{
    if (!g || !g->exec) return fail(ZS_EINVAL, "graph is null");
    HIP_TRY(hipGraphLaunch(g->exec, stream));
    return ZS_OK;
}

zs_status zs_release_workspaces(hipStream_t stream)
{
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    StoreWork *sw = nullptr;
    QueryWork *qw = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_swmu);
        auto it = g_sw.find({device, stream});
        if (it != g_sw.end()) sw = it->second;
    }
    {
        std::lock_guard<std::mutex> lk(g_qwmu);
        auto it = g_qw.find({device, stream});
        if (it != g_qw.end()) qw = it->second;
    }
    // The entries stay in their maps (a call that has already looked one up
    // may be waiting on its lock); only their memory is returned, and it
    // grows again on the next call on the stream.
    if (sw) {
        std::lock_guard<std::mutex> lk(sw->mu);
        HIP_TRY(hipStreamSynchronize(stream));
        sw->release();
    }
    if (qw) {
        std::lock_guard<std::recursive_mutex> lk(qw->mu);
        HIP_TRY(hipStreamSynchronize(stream));
        qw->w.release();
    }
    return ZS_OK;
}

void zs_store_free(zs_store *st)
{
    if (!st) return;
    (void)hipDeviceSynchronize();
    if (st->base) (void)hipFree(st->base);
    delete st;
}

int64_t zs_store_bytes(const zs_store *st)
{
    if (!st) return 0;
    return (int64_t)st->esize() * (st->t * st->k + st->nb * st->k * st->c) +
           (int64_t)sizeof(double) * (st->nb * st->k + 2 * st->n2 * st->c * st->c) +
           (int64_t)sizeof(int32_t) * st->nb;
}

zs_status zs_store_info(const zs_store *st, int64_t *t, int64_t *c, int64_t *b, int32_t *k,
                        int64_t *nb, int32_t *mode)
{
    if (!st) return fail(ZS_EINVAL, "store is null");
    if (t) *t = st->t;
    if (c) *c = st->c;
    if (b) *b = st->b;
    if (k) *k = st->k;
    if (nb) *nb = st->nb;
    if (mode) *mode = (int32_t)st->mode;
    return ZS_OK;
}

zs_status zs_store_get_block(const zs_store *st, int64_t i, void *U, double *S, void *V,
                             int32_t *k_i, hipStream_t stream)
{
    if (!st) return fail(ZS_EINVAL, "store is null");
    if (i < 0 || i >= st->nb) return fail(ZS_ERANGE, "block %lld outside [0, %lld)", (long long)i,
                                          (long long)st->nb);
    if (!U || !S || !V || !k_i) return fail(ZS_EINVAL, "null output pointer");
    const int64_t rows = st->block_rows(i), k = st->k, c = st->c;
    const size_t es = st->esize();
    const char *Us = static_cast<const char *>(st->U), *Vs = static_cast<const char *>(st->Vt);
    HIP_TRY(hipMemcpyAsync(U, Us + i * st->b * k * es, es * rows * k, hipMemcpyDeviceToDevice,
                           stream));
    HIP_TRY(hipMemcpyAsync(S, st->S + i * k, sizeof(double) * k, hipMemcpyDeviceToDevice, stream));
    // V_(i) = (V_(i)^T)^T: c x k from the stored k x c rows.
    for (int64_t j = 0; j < k; ++j)
        HIP_TRY(hipMemcpy2DAsync(static_cast<char *>(V) + j * es, es * k, Vs + (i * k + j) * c * es,
                                 es, es, c, hipMemcpyDeviceToDevice, stream));
    HIP_TRY(hipMemcpyAsync(k_i, st->kvec + i, sizeof(int32_t), hipMemcpyDeviceToDevice, stream));
    return ZS_OK;
}

zs_status zs_sync_status(const zs_store *cst, hipStream_t stream)
{
    if (!cst) return fail(ZS_EINVAL, "store is null");
    HIP_TRY(hipStreamSynchronize(stream));
    int conv = 0;
    HIP_TRY(hipMemcpy(&conv, cst->conv, sizeof(int), hipMemcpyDeviceToHost));
    if (conv) {
        int zero = 0;
        HIP_TRY(hipMemcpy(cst->conv, &zero, sizeof(int), hipMemcpyHostToDevice));
        return fail(ZS_ENOCONV, "an eigen-solve hit the sweep cap");
    }
    return ZS_OK;
}

zs_status zs_set_sweep_cap(int cap)
{
    if (cap < 1) return fail(ZS_EINVAL, "sweep cap %d < 1", cap);
    HIP_TRY(set_sweep_cap(cap));
    return ZS_OK;
}

void zs_timing_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    g_timing = on != 0;
}

void zs_timing_reset(void)
{
    std::lock_guard<std::mutex> lk(g_tmu);
    for (auto &p : g_pending) {
        (void)hipEventSynchronize(p.b);
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    g_pending.clear();
    g_acc.clear();
}

zs_status zs_timing_get(const char *name, int64_t *launches, double *total_ms)
{
    if (!name) return fail(ZS_EINVAL, "name is null");
    std::lock_guard<std::mutex> lk(g_tmu);
    for (auto &p : g_pending) {
        HIP_TRY(hipEventSynchronize(p.b));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, p.a, p.b));
        auto &acc = g_acc[p.name];
        acc.first += 1;
        acc.second += ms;
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    g_pending.clear();
    auto it = g_acc.find(name);
    if (launches) *launches = it == g_acc.end() ? 0 : it->second.first;
    if (total_ms) *total_ms = it == g_acc.end() ? 0.0 : it->second.second;
    return ZS_OK;
}

}  // extern "C"
