// Host half of the query plan (Alg. 3 index math), shared by the runtime and
// host-only checks.  `Store` needs b, t, n2 (leaves of the Gram tree), f32 and
// block_rows(i); no HIP headers.
#pragma once

#include <stdint.h>

#include <cstring>
#include <vector>

#include "zs_types.h"

namespace zs {

// The O(1) part of the plan of one query (Alg. 3 index math, host side).
// Pieces are the touched blocks S..E; boundary blocks cut by the range go
// through the Partial-SVD.  Whole blocks form one contiguous run whose Gram
// comes from the Gram tree.  Fills the query's descriptor `d` and problem
// `pr`, reports its Partial-SVD pieces, their stack-row slots and its tree
// nodes to `sink`, and advances `slot` past its projection chunks (chunk j
// is make_stack_chunk(j, ...)).  Every quantity depends only on this query
// and on where the batch puts it (piece0, y0, c0, the first slot).
template <class Store, class Sink>
void plan_one(const Store *st, int32_t q, int64_t ts, int64_t te, int32_t kq, int64_t u_off,
              int64_t ldu, double *s_dst, void *v_dst, int64_t ldv, int32_t *k_dst,
              int64_t piece0, int64_t y0, int64_t c0, int32_t &slot, Sink &sink, QueryDesc &d,
              Prob &pr)
{
    (void)q;
    const int64_t b = st->b;
    const int64_t S_ = ts / b, E_ = (te - 1) / b;
    const int64_t lo = ts - S_ * b, hi = te - E_ * b;
    const int64_t np = E_ - S_ + 1;
    std::memset(&d, 0, sizeof d);
    d.S = S_;
    d.ts = ts;
    d.piece0 = piece0;
    d.y0 = y0;
    d.c0 = c0;
    d.u_off = u_off;
    d.ldu = ldu;
    d.np = (int32_t)np;
    d.lo = (int32_t)lo;
    d.hi = (int32_t)hi;
    d.kq = kq;
    d.t0 = sink.npidx();
    // first piece: rows [lo, np == 1 ? hi : rows_S); last piece (np > 1): [0, hi)
    const bool first_partial = lo != 0 || (np == 1 ? hi != st->block_rows(S_) : false);
    const bool last_partial = np > 1 && hi != st->block_rows(E_);
    d.first_partial = first_partial ? 1 : 0;
    std::memset(&pr, 0, sizeof pr);
    pr.m0 = sink.nmsrc();
    if (first_partial) {
        sink.add_msrc(sink.npidx());
        sink.add_pidx((int32_t)piece0);
    }
    if (last_partial) {
        sink.add_msrc(sink.npidx());
        sink.add_pidx((int32_t)(piece0 + np - 1));
    }
    pr.nm = sink.nmsrc() - pr.m0;
    // Whole blocks [whole_a, whole_e) are contiguous: cover them with tree nodes.
    const int64_t whole_a = S_ + (first_partial ? 1 : 0);
    const int64_t whole_e = E_ + 1 - (last_partial ? 1 : 0);
    pr.g0 = sink.ngsrc();
    if (whole_a < whole_e) {
        int64_t l = whole_a + st->n2, r = whole_e + st->n2;
        while (l < r) {
            if (l & 1) sink.add_gsrc(l++);
            if (r & 1) sink.add_gsrc(--r);
            l >>= 1;
            r >>= 1;
        }
    }
    pr.ng = sink.ngsrc() - pr.g0;
    pr.y0 = slot;
    slot += (int32_t)((np + kQueryChunkPieces - 1) / kQueryChunkPieces);
    pr.ny = slot - pr.y0;
    pr.kk = kq;
    pr.v_dst = v_dst;
    pr.v_f32 = st->f32;
    pr.v_rs = ldv;
    pr.v_cs = 1;
    pr.s_dst = s_dst;
    pr.k_dst = k_dst;
}

// Sink of plan_one for a batch: growable host arrays.
struct VecSink {
    std::vector<int32_t> pidx;          // pieces that need a Partial-SVD
    std::vector<int32_t> msrc;          // Partial-SVD slots of the problems' stack rows
    std::vector<int64_t> gsrc;          // tree node indices
    int32_t npidx() const { return (int32_t)pidx.size(); }
    int32_t nmsrc() const { return (int32_t)msrc.size(); }
    int32_t ngsrc() const { return (int32_t)gsrc.size(); }
    void add_pidx(int32_t v) { pidx.push_back(v); }
    void add_msrc(int32_t v) { msrc.push_back(v); }
    void add_gsrc(int64_t v) { gsrc.push_back(v); }
};

// Sink of plan_one for one query planned into a SinglePlan (fixed arrays).
struct PlanSink {
    SinglePlan &p;
    bool overflow = false;
    int32_t nm = 0;
    int32_t npidx() const { return p.npidx; }
    int32_t nmsrc() const { return nm; }
    int32_t ngsrc() const { return p.ngsrc; }
    void add_pidx(int32_t v)
    {
        if (p.npidx < 2) p.pidx[p.npidx++] = v;
        else overflow = true;
    }
    void add_msrc(int32_t v)
    {
        if (nm < 2) p.msrc[nm++] = v;
        else overflow = true;
    }
    void add_gsrc(int64_t v)
    {
        if (p.ngsrc < kMaxPlanNodes) p.gsrc[p.ngsrc++] = v;
        else overflow = true;
    }
};

}  // namespace zs
