// Host-only check of the query planner (plan.h: the Alg. 3 index math of one
// query), built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_sanitizers.py.  For random block sizes, series lengths (with
// short last blocks) and ranges, the planner's descriptor, Partial-SVD pieces
// and Gram-tree nodes are compared with an enumeration of the range's rows:
// the touched blocks, the rows kept of each, which blocks are cut, and the
// whole blocks covered by the tree nodes exactly once.
#include "plan.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <set>
#include <vector>

namespace {

struct HostStore {
    int64_t t, b, n2;
    int32_t f32;
    int64_t block_rows(int64_t i) const { return std::min(b, t - i * b); }
};

uint64_t g_state = 0x9E3779B97F4A7C15ull;
uint64_t next()
{
    g_state ^= g_state << 13;
    g_state ^= g_state >> 7;
    g_state ^= g_state << 17;
    return g_state;
}
int64_t uniform(int64_t lo, int64_t hi) { return lo + (int64_t)(next() % (uint64_t)(hi - lo + 1)); }

int g_fail = 0;
void check(bool ok, const char *what, int64_t t, int64_t b, int64_t ts, int64_t te)
{
    if (ok) return;
    if (g_fail < 20) std::printf("FAIL %s: t=%lld b=%lld [%lld, %lld)\n", what, (long long)t,
                                 (long long)b, (long long)ts, (long long)te);
    ++g_fail;
}

// Leaves [first, last) under node x of a tree with n2 leaves (leaf i is node n2 + i).
void leaves_of(int64_t x, int64_t n2, int64_t &first, int64_t &last)
{
    int64_t lo = x, hi = x + 1;
    while (lo < n2) {
        lo *= 2;
        hi *= 2;
    }
    first = lo - n2;
    last = hi - n2;
}

}  // namespace

int main()
{
    int cases = 0;
    for (int trial = 0; trial < 4000; ++trial) {
        HostStore st;
        st.b = uniform(1, 64);
        st.t = uniform(1, 40 * st.b + 7);
        const int64_t nb = (st.t + st.b - 1) / st.b;
        st.n2 = 1;
        while (st.n2 < nb) st.n2 *= 2;
        st.f32 = (int32_t)(trial & 1);
        zs::VecSink sink;
        int32_t slot = (int32_t)uniform(0, 5);
        // a few queries planned into one batch, as the runtime does
        int64_t piece0 = 0;
        for (int q = 0; q < 4; ++q) {
            const int64_t ts = uniform(0, st.t - 1), te = uniform(ts + 1, st.t);
            const int32_t kq = (int32_t)uniform(1, 8);
            const int32_t slot0 = slot;
            const size_t p0 = sink.pidx.size(), g0 = sink.gsrc.size();
            zs::QueryDesc d;
            zs::Prob pr;
            double s_dummy[8];
            int32_t k_dummy = 0;
            zs::plan_one(&st, q, ts, te, kq, 0, kq, s_dummy, nullptr, kq, &k_dummy, piece0, 0, 0,
                         slot, sink, d, pr);
            // enumeration of the rows
            const int64_t S = ts / st.b, E = (te - 1) / st.b, np = E - S + 1;
            check(d.S == S && d.np == np, "touched blocks", st.t, st.b, ts, te);
            std::set<int64_t> cut, whole;
            for (int64_t i = S; i <= E; ++i) {
                const int64_t r0 = std::max(ts, i * st.b) - i * st.b;
                const int64_t r1 = std::min(te, i * st.b + st.block_rows(i)) - i * st.b;
                check(r0 < r1, "empty piece", st.t, st.b, ts, te);
                if (i == S) check(d.lo == r0, "first row kept", st.t, st.b, ts, te);
                if (i == E) check(d.hi == r1, "last row kept", st.t, st.b, ts, te);
                if (r0 != 0 || r1 != st.block_rows(i)) cut.insert(i);
                else whole.insert(i);
            }
            check(cut.size() <= 2, "at most two cut blocks", st.t, st.b, ts, te);
            check(d.first_partial == (cut.count(S) ? 1 : 0), "first piece cut", st.t, st.b, ts, te);
            // Partial-SVD pieces: exactly the cut blocks, in order, with their slots
            std::set<int64_t> planned_cut;
            for (size_t i = p0; i < sink.pidx.size(); ++i) {
                planned_cut.insert(S + (sink.pidx[i] - piece0));
                check(sink.msrc[pr.m0 + (i - p0)] == (int32_t)i, "stack-row slot", st.t, st.b, ts, te);
            }
            check(planned_cut == cut, "cut blocks", st.t, st.b, ts, te);
            check(pr.nm == (int32_t)cut.size() && d.t0 == (int32_t)p0, "Partial-SVD slots", st.t,
                  st.b, ts, te);
            // tree nodes: the whole blocks, each once, no more than 2 per level
            std::vector<int> seen(st.n2, 0);
            for (size_t i = g0; i < sink.gsrc.size(); ++i) {
                const int64_t x = sink.gsrc[i];
                check(x >= 1 && x < 2 * st.n2, "node index", st.t, st.b, ts, te);
                if (x < 1 || x >= 2 * st.n2) continue;
                int64_t f, l;
                leaves_of(x, st.n2, f, l);
                for (int64_t j = f; j < l; ++j) ++seen[j];
            }
            for (int64_t j = 0; j < st.n2; ++j)
                check(seen[j] == (whole.count(j) ? 1 : 0), "whole blocks covered once", st.t, st.b, ts, te);
            int levels = 0;
            for (int64_t v = st.n2; v > 1; v /= 2) ++levels;
            check(pr.ng == (int32_t)(sink.gsrc.size() - g0) && pr.ng <= 2 * levels + 2, "node count",
                  st.t, st.b, ts, te);
            // projection chunks: ceil(np / 32) slots, covering the pieces once
            check(pr.y0 == slot0 && pr.ny == slot - slot0 &&
                      pr.ny == (int32_t)((np + zs::kQueryChunkPieces - 1) / zs::kQueryChunkPieces),
                  "chunk slots", st.t, st.b, ts, te);
            int64_t covered = 0;
            for (int32_t j = 0; j < pr.ny; ++j) {
                const zs::StackChunk ch = zs::make_stack_chunk(j, (int32_t)np, 4, kq, 0, piece0, q, slot0 + j);
                check(ch.piece0 == piece0 + covered && ch.npieces > 0, "chunk pieces", st.t, st.b, ts, te);
                covered += ch.npieces;
            }
            check(covered == np, "chunks cover the pieces", st.t, st.b, ts, te);
            check(pr.kk == kq && pr.k_dst == &k_dummy && pr.s_dst == s_dummy, "problem outputs",
                  st.t, st.b, ts, te);
            piece0 += np;
            ++cases;
        }
    }
    // the fixed-capacity sink of the single-query path flags overflow instead of writing past
    zs::SinglePlan p;
    std::memset(&p, 0, sizeof p);
    zs::PlanSink ps{p};
    for (int i = 0; i < zs::kMaxPlanNodes + 5; ++i) ps.add_gsrc(i);
    check(ps.overflow && p.ngsrc == zs::kMaxPlanNodes, "fixed sink overflow", 0, 0, 0, 0);
    if (g_fail) {
        std::printf("plan_check: %d failures in %d cases\n", g_fail, cases);
        return 1;
    }
    std::printf("plan_check ok %d cases\n", cases);
    return 0;
}
