"""The serving loop on the GPU: every served query equals the same query run
alone (bitwise), under small budgets that force several batches with two
batches in flight on two streams, and a seeded sample of served results
matches the oracle's query phase on the downloaded store."""
import numpy as np
import pytest
import torch

from paper_1805_00754_amd import serve, synth
from paper_1805_00754_amd import zoomsvd as zs
import oracle
from tests.gpu_common import (F32_KW, RANK_TOL_F32, compare_svd, download_store, mode_tol, say,
                              to_dev)

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("max_queries,budget,rate,mode", [
    (16, 1536 << 10, 20000.0, "fp64"),
    (64, 64 << 20, 4000.0, "fp64"),
    (16, 512 << 10, 20000.0, "fp32"),
])
def test_served_equals_single(max_queries, budget, rate, mode):
    zs.load()
    ser, cfg = synth.workload("sinmix_10k_x64_f64")
    if mode == "fp64":
        st = zs.zs_store_blocks(to_dev(ser.A), cfg["b"], cfg["k"])
    else:
        st = zs.zs_store_blocks(to_dev(ser.A, torch.float32), cfg["b"], cfg["k"],
                                mode=zs.ZS_MODE_FP32)
    esize = 8 if mode == "fp64" else 4
    torch.cuda.synchronize()
    rng = synth.rng_for(77)
    reqs = serve.make_requests(rng, st.t, 120, rate, 150, 8000, [3, 10])
    # one request too large for the budget is rejected, not served
    big = serve.Request(len(reqs), 0, st.t, cfg["k"], reqs[-1].arrival + 1e-4)
    reqs.append(big)
    srv = serve.Server(st, max_queries=max_queries, budget_bytes=budget)
    got = {}

    def on_batch(info, arena, sarena, kout):
        for q, r in enumerate(info["batch"]):
            n = r.t_e - r.t_s
            U = arena[info["u_off"][q]:info["u_off"][q] + n * r.k_q].view(n, r.k_q)
            S = sarena[info["s_off"][q]:info["s_off"][q] + r.k_q]
            V = arena[info["v_off"][q]:info["v_off"][q] + st.c * r.k_q].view(st.c, r.k_q)
            got[r.idx] = (U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy(), int(kout[q].item()))

    say("serve", max_queries, budget, rate)
    res = srv.run(reqs, on_batch=on_batch)
    # admission counts each request's outputs and the library's scratch for it
    too_big = {r.idx for r in reqs if srv.policy.bytes_of(r) > budget}
    for r in reqs[:5]:
        assert srv.policy.bytes_of(r) == (serve.output_bytes(r.t_e - r.t_s, r.k_q, st.c, esize)
                                          + zs.zs_query_scratch_bytes(st, r.t_s, r.t_e, r.k_q))
        assert zs.zs_query_scratch_bytes(st, r.t_s, r.t_e, r.k_q) > 0
    assert set(res["rejected"]) == too_big
    assert big.idx in too_big or budget > (1 << 20)
    assert sum(res["batches"]) == len(got)
    assert max(res["batches"]) <= max_queries
    for r in reqs:
        if r.idx in res["rejected"]:
            continue
        U, S, V, ko = zs.zs_query(st, r.t_s, r.t_e, r.k_q)
        torch.cuda.synchronize()
        gU, gS, gV, gk = got[r.idx]
        assert gk == int(ko.item())
        np.testing.assert_array_equal(gS, S.cpu().numpy())
        np.testing.assert_array_equal(gV, V.cpu().numpy())
        np.testing.assert_array_equal(gU, U.cpu().numpy())
        assert res["latency"][r.idx] > 0
    assert len(res["batch_ms"]) == len(res["batches"])
    # a seeded sample of served results against the oracle's query phase on
    # the store downloaded from the GPU
    Ug, Sg, Vg, kg = download_store(st)
    f64 = mode == "fp64"
    ost = oracle.store_from_arrays(st.t, st.c, st.b, st.k, Ug, Sg, Vg, kg,
                                   **({} if f64 else dict(rank_tol=RANK_TOL_F32)))
    served_ids = sorted(got)
    pick = synth.rng_for(78).choice(len(served_ids), size=min(12, len(served_ids)), replace=False)
    for i in pick:
        r = reqs[served_ids[i]]
        gU, gS, gV, gk = got[r.idx]
        compare_svd((gU.astype(np.float64), gS, gV.astype(np.float64), gk),
                    oracle.query(ost, r.t_s, r.t_e, r.k_q),
                    mode_tol(zs.ZS_MODE_FP64 if f64 else zs.ZS_MODE_FP32), st.c,
                    "served [%d, %d)" % (r.t_s, r.t_e), **({} if f64 else F32_KW))
