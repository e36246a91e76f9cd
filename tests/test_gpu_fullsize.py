"""Parity at the benchmark's full size, in the launch configuration bench.py
times: the 10^6 x 128 FP64 series (b = 1000, k = 20) stored in one call and
the 1,024-query batch of 320,000-row ranges answered in one zs_query_batch.
The oracle checks a sample it can compute one by one: blocks of the store
against its storage phase, and queries of the batch against its query phase
run on the downloaded store (decoupled parity, as in test_gpu_parity)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1805_00754_amd import synth
from paper_1805_00754_amd import zoomsvd as zs
from tests.gpu_common import TOL_FP64, compare_svd, download_store, say, to_dev

pytestmark = pytest.mark.gpu

WORKLOAD = "sinmix_1m_x128_f64"
QUERIES, QUERY_LEN = 1024, 320_000


@pytest.fixture(scope="module")
def full():
    zs.load()
    oracle.load()
    say("full size: generating", WORKLOAD)
    ser, cfg = synth.workload(WORKLOAD)
    t = ser.A.shape[0]
    ts, te = synth.queries_fixed(ser.rng, t, QUERIES, QUERY_LEN)   # the benchmark's queries
    kq = np.full(QUERIES, cfg["k"], np.int32)
    A = to_dev(ser.A)
    say("full size: store and batch")
    st = zs.zs_store_blocks(A, cfg["b"], cfg["k"])
    out = zs.zs_query_batch(st, ts, te, kq)
    zs.zs_sync_status(st)
    torch.cuda.synchronize()
    del A
    say("full size: downloading the store")
    U, S, V, kk = download_store(st)
    ost = oracle.store_from_arrays(st.t, st.c, st.b, st.k, U, S, V, kk)
    yield ser.A, cfg, st, out, ts, te, (U, S, V, kk), ost
    del out
    st.free()
    torch.cuda.empty_cache()


def test_fullsize_store_sample(full):
    A, cfg, st, out, ts, te, (U, S, V, kk), ost = full
    b, k = cfg["b"], cfg["k"]
    rng = synth.rng_for(1805)
    blocks = sorted(set(rng.integers(0, st.nb, size=6).tolist()) | {0, st.nb - 1})
    for i in blocks:
        r = st.block_rows(i)
        ref = oracle.store(np.ascontiguousarray(A[i * b:i * b + r]), b, k)
        got = (U[i * b:i * b + r], S[i], V[i], int(kk[i]))
        say("full size: block", i)
        compare_svd(got, (ref.U[:r], ref.S[0], ref.V[0], int(ref.k_i[0])), TOL_FP64, st.c,
                    "block %d" % i)


def test_fullsize_batch_all_sigma_v(full):
    """Sigma, V and k_out of every query of the batch against the oracle's
    query phase on the downloaded store (Alg. 2; U is checked on a sample)."""
    A, cfg, st, out, ts, te, _, ost = full
    say("full size: oracle sigma and V of all %d queries" % QUERIES)
    refs = oracle.query_batch(ost, ts, te, cfg["k"], with_u=False)
    S_all = out.S.cpu().numpy()
    V_all = out.V.cpu().numpy()
    k_all = out.k_out.cpu().numpy()
    for q in range(QUERIES):
        so, vo = int(out.s_off[q]), int(out.v_off[q])
        kq = int(out.k_q[q])
        got = (None, S_all[so:so + kq], V_all[vo:vo + st.c * kq].reshape(st.c, kq), int(k_all[q]))
        compare_svd(got, refs[q], TOL_FP64, st.c, "query %d [%d,%d)" % (q, ts[q], te[q]))


def test_fullsize_batch_sample(full):
    """U of a seeded sample of 32 queries (Eq. (9)), with the joint signs of
    (u_j, v_j); three of them also alone, bitwise equal to the batch."""
    A, cfg, st, out, ts, te, _, ost = full
    rng = synth.rng_for(1806)
    sample = sorted(set(rng.choice(QUERIES, size=29, replace=False).tolist())
                    | {0, QUERIES // 2, QUERIES - 1})
    refs = oracle.query_batch(ost, ts[sample], te[sample], cfg["k"])
    for ref, q in zip(refs, sample):
        Ub, Sb, Vb, kb = out.result(q)
        got = (Ub.cpu().numpy(), Sb.cpu().numpy(), Vb.cpu().numpy(), int(kb.item()))
        say("full size: query", q, int(ts[q]), int(te[q]))
        compare_svd(got, ref, TOL_FP64, st.c, "query %d [%d,%d)" % (q, ts[q], te[q]))
        if q not in (0, QUERIES // 2, QUERIES - 1):
            continue
        # the same query alone gives the batch's bits
        U1, S1, V1, k1 = zs.zs_query(st, int(ts[q]), int(te[q]), cfg["k"])
        torch.cuda.synchronize()
        assert int(k1.item()) == got[3]
        np.testing.assert_array_equal(S1.cpu().numpy(), got[1])
        np.testing.assert_array_equal(V1.cpu().numpy(), got[2])
        np.testing.assert_array_equal(U1.cpu().numpy(), got[0])
