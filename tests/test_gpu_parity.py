"""GPU parity of the HIP path against the CPU oracle (FP64 mode).

Decoupled, as the storage phase's truncation is not unique when two singular
values of a block tie at the cut: (1) store parity block by block against
the oracle's storage phase; (2) query parity by running the oracle's query
phase on the store downloaded from the GPU; (3) end-to-end against the
direct SVD of the raw rows on block-rank-<=k data, where the method is exact.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1805_00754_amd import synth
from paper_1805_00754_amd import zoomsvd as zs
from tests.gpu_common import TOL_FP64, compare_svd, download_store, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    zs.load()
    oracle.load()


def gpu_store(A, b, k):
    st = zs.zs_store_blocks(to_dev(A), b, k)
    torch.cuda.synchronize()
    return st


def gpu_query(st, ts, te, kq):
    U, S, V, ko = zs.zs_query(st, ts, te, kq)
    zs.zs_sync_status(st)       # raises on an eigen-solve that hit its sweep cap
    return U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy(), int(ko.item())


def check_store(A, b, k, what):
    say("store parity", what, A.shape, "b", b, "k", k)
    st = gpu_store(A, b, k)
    Ug, Sg, Vg, kg = download_store(st)
    ost = oracle.store(A, b, k)
    c = A.shape[1]
    for i in range(st.nb):
        r = st.block_rows(i)
        got = (Ug[i * b:i * b + r], Sg[i], Vg[i], int(kg[i]))
        ref = (ost.U[i * b:i * b + r], ost.S[i], ost.V[i], int(ost.k_i[i]))
        compare_svd(got, ref, TOL_FP64, c, "%s block %d" % (what, i))
    return st, (Ug, Sg, Vg, kg)


# ------------------------------------------------------------------ storage
@pytest.mark.parametrize("t,c,b,k", [(10_000, 64, 100, 10), (21_100, 128, 1000, 20),
                                     (3_050, 9, 128, 4), (700, 33, 64, 33), (50, 16, 100, 8)])
def test_store_parity_sinmix(t, c, b, k):
    ser = synth.sinusoid_mixture(t, c, sources=min(8, c), seed=7 + c, noise="iid", noise_sigma=0.1)
    check_store(ser.A, b, k, "sinmix %dx%d" % (t, c))


def test_store_parity_rank_deficient_and_zero_block():
    t, c, b, k = 1_000, 24, 100, 6
    A = synth.block_low_rank(t, c, b, rank=3, seed=5)
    A[300:400] = 0.0                  # an all-zero block
    st, (Ug, Sg, Vg, kg) = check_store(A, b, k, "rank3")
    assert kg[3] == 0 and np.all(Sg[3] == 0)
    assert all(kg[i] == 3 for i in range(st.nb) if i != 3)


# ------------------------------------------------------------------ queries
QUERY_RANGES = [(0, 10_000), (37, 9_963), (100, 200), (150, 151), (199, 201), (4_321, 4_399),
                (5_000, 5_100), (0, 1), (9_999, 10_000), (250, 8_250)]


@pytest.fixture(scope="module")
def sinmix64():
    ser, cfg = synth.workload("sinmix_10k_x64_f64")
    st = gpu_store(ser.A, cfg["b"], cfg["k"])
    U, S, V, kk = download_store(st)
    ost = oracle.store_from_arrays(st.t, st.c, st.b, st.k, U, S, V, kk)
    return ser.A, cfg, st, ost


@pytest.mark.parametrize("rng", QUERY_RANGES)
@pytest.mark.parametrize("kq", [10, 3])
def test_query_parity_on_gpu_store(sinmix64, rng, kq):
    A, cfg, st, ost = sinmix64
    ts, te = rng
    say("query parity", ts, te, kq)
    got = gpu_query(st, ts, te, kq)
    ref = oracle.query(ost, ts, te, kq)
    compare_svd(got, ref, TOL_FP64, st.c, "query [%d,%d) kq %d" % (ts, te, kq))


# Stores of other widths and ranks: every compiled width of the block product
# and of the stack projection (k rounded up to 4, 8, 12, ..., 32, 48, 64).
OTHER_STORES = [(3_000, 128, 250, 20), (2_000, 33, 64, 33), (1_500, 64, 100, 64), (1_200, 9, 50, 4),
                (1_700, 30, 128, 27), (900, 16, 40, 13)]


@pytest.mark.parametrize("t,c,b,k", OTHER_STORES)
def test_query_parity_other_widths(t, c, b, k):
    ser = synth.sinusoid_mixture(t, c, sources=min(6, c), seed=31 + k, noise="iid",
                                 noise_sigma=0.1)
    st = gpu_store(ser.A, b, k)
    U, S, V, kk = download_store(st)
    ost = oracle.store_from_arrays(st.t, st.c, st.b, st.k, U, S, V, kk)
    rng = synth.rng_for(40 + k)
    ts, te = synth.queries_uniform(rng, t, 4, 1, t)
    for q, kq in enumerate([k, 1, max(1, k // 2), max(1, k - 1)]):
        say("query parity", (t, c, b, k), int(ts[q]), int(te[q]), kq)
        got = gpu_query(st, int(ts[q]), int(te[q]), kq)
        ref = oracle.query(ost, int(ts[q]), int(te[q]), kq)
        compare_svd(got, ref, TOL_FP64, c, "c %d k %d [%d,%d) kq %d" % (c, k, ts[q], te[q], kq))


# c above 128: the eigen-solver keeps its matrix in global scratch and the
# leaf Grams go through the Gram kernel.
LARGE_C = [(3_000, 200, 600, 24), (4_000, 256, 1000, 32), (2_600, 512, 1300, 48),
           (2_100, 1024, 1050, 64),
           # short last blocks (300 rows) at c = 256 and c = 1024
           (3_300, 256, 1000, 32), (2_300, 1024, 1000, 64),
           # the first width of each form of the solver (c = 129, 257, 513):
           # trailing blocks of one element past a 64-column chunk
           (2_100, 129, 700, 16), (2_200, 257, 900, 40), (2_200, 513, 1100, 20)]


@pytest.mark.parametrize("t,c,b,k", LARGE_C)
def test_large_c_store_and_query_parity(t, c, b, k):
    ser = synth.sinusoid_mixture(t, c, sources=12, seed=5 + c, noise="iid", noise_sigma=0.1)
    st, (U, S, V, kk) = check_store(ser.A, b, k, "large c %d" % c)
    gst = oracle.store_from_arrays(st.t, st.c, st.b, st.k, U, S, V, kk)
    rng = synth.rng_for(c)
    ts, te = synth.queries_uniform(rng, t, 4, 1, t)
    for q in range(4):
        kq = [k, 5][q % 2]
        say("large c query", c, int(ts[q]), int(te[q]), kq)
        got = gpu_query(st, int(ts[q]), int(te[q]), kq)
        ref = oracle.query(gst, int(ts[q]), int(te[q]), kq)
        compare_svd(got, ref, TOL_FP64, c, "c %d [%d,%d) kq %d" % (c, ts[q], te[q], kq))


# Block sizes of the paper's sensitivity study (Sec. 4.5, Fig. 6) beyond the
# default 10^3: 10 (fewer rows per block than the rank k, so k_i = 10), 10^4
# and 10^5 rows per block, each with a short last block.
@pytest.mark.parametrize("t,c,b,k", [(2_003, 128, 10, 20), (25_000, 128, 10_000, 20),
                                     (230_000, 128, 100_000, 20)])
def test_large_block_sizes(t, c, b, k):
    ser = synth.sinusoid_mixture(t, c, sources=16, seed=61 + b // 1000, noise="ar1",
                                 noise_sigma=0.05)
    st, (U, S, V, kk) = check_store(ser.A, b, k, "b %d" % b)
    gst = oracle.store_from_arrays(st.t, st.c, st.b, st.k, U, S, V, kk)
    rng = synth.rng_for(b)
    ts, te = synth.queries_loguniform(rng, t, 4, min(1e3, t // 4), t)
    for q in range(4):
        kq = [k, 7][q % 2]
        say("b %d query" % b, int(ts[q]), int(te[q]), kq)
        got = gpu_query(st, int(ts[q]), int(te[q]), kq)
        ref = oracle.query(gst, int(ts[q]), int(te[q]), kq)
        compare_svd(got, ref, TOL_FP64, c, "b %d [%d,%d) kq %d" % (b, ts[q], te[q], kq))
    st.free()


def test_query_exact_on_block_low_rank():
    """Block rank <= k: the stitched SVD equals the direct SVD of A[t_s:t_e)."""
    t, c, b, k = 5_300, 40, 100, 6
    A = synth.block_low_rank(t, c, b, rank=5, seed=9)
    st = gpu_store(A, b, k)
    for ts, te in [(0, 5_300), (37, 4_563), (120, 180), (99, 101), (200, 300), (5_250, 5_300)]:
        say("exact", ts, te)
        got = gpu_query(st, ts, te, k)
        ref = oracle.direct(A, ts, te, k)
        compare_svd(got, ref, TOL_FP64, c, "exact [%d,%d)" % (ts, te))


def test_rank_one_closed_form():
    t, c, b = 4_000, 12, 256
    A, s_vec, m = synth.rank_one(t, c, seed=3)
    st = gpu_store(A, b, 4)
    for ts, te in [(0, 4_000), (10, 3_900), (256, 512), (255, 257), (3_999, 4_000)]:
        U, S, V, ko = gpu_query(st, ts, te, 4)
        assert ko == 1
        np.testing.assert_allclose(S[0], np.linalg.norm(s_vec[ts:te]) * np.linalg.norm(m),
                                   rtol=1e-12)
        assert np.all(S[1:] == 0)
        u = s_vec[ts:te] / np.linalg.norm(s_vec[ts:te])
        assert abs(abs(U[:, 0] @ u) - 1) < 1e-12
        assert abs(abs(V[:, 0] @ (m / np.linalg.norm(m))) - 1) < 1e-12


def test_short_matrix_single_short_block():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((37, 20))
    st = gpu_store(A, 100, 8)
    got = gpu_query(st, 3, 30, 8)
    ost = oracle.store(A, 100, 8)
    ref = oracle.query(ost, 3, 30, 8)
    compare_svd(got, ref, TOL_FP64, 20, "short")


# ------------------------------------------------------------------ batching
def test_batch_equals_single_bitwise(sinmix64):
    A, cfg, st, ost = sinmix64
    rng = synth.rng_for(11)
    ts, te = synth.queries_uniform(rng, st.t, 40, 150, 8_000)
    kq = rng.integers(1, st.k + 1, size=40).astype(np.int32)
    batch = zs.zs_query_batch(st, ts, te, kq)
    torch.cuda.synchronize()
    for q in range(len(ts)):
        Ub, Sb, Vb, kb = [x.cpu().numpy() for x in batch.result(q)]
        Us, Ss, Vs, ks = gpu_query(st, int(ts[q]), int(te[q]), int(kq[q]))
        assert int(kb[0]) == ks
        np.testing.assert_array_equal(Sb, Ss)
        np.testing.assert_array_equal(Vb, Vs)
        np.testing.assert_array_equal(Ub, Us)


def test_strided_outputs_equal_dense(sinmix64):
    """Outputs with leading dimensions above k_q (column slices of wider
    tensors) hold the same values as dense outputs; the padding is untouched."""
    A, cfg, st, ost = sinmix64
    dev = torch.device("cuda", 0)
    for (ts, te, kq) in [(137, 1789, st.k), (250, 4_321, 3), (1_000, 1_100, 7)]:
        n = te - ts
        Ub = torch.full((n, kq + 5), 7.0, dtype=torch.float64, device=dev)
        Vb = torch.full((st.c, kq + 2), 7.0, dtype=torch.float64, device=dev)
        Us, Ss, Vs, ks = zs.zs_query(st, ts, te, kq, U=Ub[:, :kq], V=Vb[:, :kq])
        Ud, Sd, Vd, kd = zs.zs_query(st, ts, te, kq)
        torch.cuda.synchronize()
        assert int(ks.item()) == int(kd.item())
        np.testing.assert_array_equal(Us.cpu().numpy(), Ud.cpu().numpy())
        np.testing.assert_array_equal(Vs.cpu().numpy(), Vd.cpu().numpy())
        np.testing.assert_array_equal(Ss.cpu().numpy(), Sd.cpu().numpy())
        assert bool((Ub[:, kq:] == 7.0).all()) and bool((Vb[:, kq:] == 7.0).all())


def test_batch_matches_oracle(sinmix64):
    A, cfg, st, ost = sinmix64
    rng = synth.rng_for(12)
    ts, te = synth.queries_uniform(rng, st.t, 20, 150, 8_000)
    batch = zs.zs_query_batch(st, ts, te, st.k)
    zs.zs_sync_status(st)
    refs = oracle.query_batch(ost, ts, te, st.k)
    for q in range(len(ts)):
        got = [x.cpu().numpy() for x in batch.result(q)]
        got[3] = int(got[3][0])
        compare_svd(tuple(got), refs[q], TOL_FP64, st.c, "batch q%d" % q)


def test_sync_status_ok(sinmix64):
    A, cfg, st, ost = sinmix64
    zs.zs_query(st, 0, 500, 5)
    zs.zs_sync_status(st)


def test_bad_query_raises(sinmix64):
    A, cfg, st, ost = sinmix64
    for ts, te, kq in [(-1, 5, 2), (5, 5, 2), (0, st.t + 1, 2), (0, 10, 0), (0, 10, st.k + 1)]:
        with pytest.raises(zs.ZSError) as ei:
            zs.zs_query(st, ts, te, kq)
        assert ei.value.status == zs.ZS_ERANGE


def test_stores_share_a_stream_workspace():
    """The query scratch belongs to the (device, stream) pair, not to a store:
    batches on two stores of different shapes issued back to back on one
    stream, with no synchronisation between them, and a batch on a store built
    after the first was freed, give the same bits as each batch run alone."""
    a = synth.sinusoid_mixture(6_000, 64, sources=6, seed=21, noise="iid", noise_sigma=0.1).A
    b = synth.sinusoid_mixture(12_000, 128, sources=9, seed=22, noise="iid", noise_sigma=0.1).A
    da, db = to_dev(a), to_dev(b)
    sa, sb = zs.zs_store_blocks(da, 500, 10), zs.zs_store_blocks(db, 1_000, 20)
    rng = synth.rng_for(23)
    qa = synth.queries_uniform(rng, 6_000, 24, 100, 5_000)
    qb = synth.queries_uniform(rng, 12_000, 48, 100, 11_000)
    ka = rng.integers(1, 11, size=24).astype(np.int32)
    kb = rng.integers(1, 21, size=48).astype(np.int32)

    def host(batch):
        return [x.cpu().numpy() for x in (batch.U, batch.S, batch.V, batch.k_out)]

    say("alone: store a, then store b")
    ref_a = host(zs.zs_query_batch(sa, *qa, ka))
    torch.cuda.synchronize()
    ref_b = host(zs.zs_query_batch(sb, *qb, kb))
    torch.cuda.synchronize()
    say("interleaved on one stream")
    outs = []
    for _ in range(2):
        outs.append((zs.zs_query_batch(sa, *qa, ka), zs.zs_query_batch(sb, *qb, kb)))
    torch.cuda.synchronize()
    for oa, ob in outs:
        for x, y in zip(host(oa), ref_a):
            np.testing.assert_array_equal(x, y)
        for x, y in zip(host(ob), ref_b):
            np.testing.assert_array_equal(x, y)
    say("a store built after the first is freed")
    sa.free()
    sa2 = zs.zs_store_blocks(da, 500, 10)
    for x, y in zip(host(zs.zs_query_batch(sa2, *qa, ka)), ref_a):
        np.testing.assert_array_equal(x, y)
    sa2.free()
    sb.free()


def test_release_workspaces_then_reuse():
    """zs_release_workspaces returns a stream's scratch; stores and batches run
    on the stream afterwards give the same bits as before, and releasing a
    stream that has nothing kept (or releasing twice) is a no-op."""
    a = synth.sinusoid_mixture(8_000, 96, sources=7, seed=24, noise="iid", noise_sigma=0.1).A
    da = to_dev(a)
    rng = synth.rng_for(25)
    ts, te = synth.queries_uniform(rng, 8_000, 32, 100, 7_000)
    kq = rng.integers(1, 13, size=32).astype(np.int32)

    def run():
        st = zs.zs_store_blocks(da, 700, 12)
        out = zs.zs_query_batch(st, ts, te, kq)
        torch.cuda.synchronize()
        blk = [x.cpu().numpy() for x in zs.zs_store_get_block(st, 5)]
        res = [x.cpu().numpy() for x in (out.U, out.S, out.V, out.k_out)] + blk
        st.free()
        return res

    say("before release")
    ref = run()
    zs.zs_release_workspaces()
    zs.zs_release_workspaces()
    say("after release")
    for x, y in zip(run(), ref):
        np.testing.assert_array_equal(x, y)
    side = torch.cuda.Stream()
    zs.zs_release_workspaces(side)            # nothing kept for this stream
