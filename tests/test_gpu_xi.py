"""The energy threshold of Eq. (1) on the GPU (zs_store_blocks_xi): the ranks
each low-rank step keeps and the kept triplets against the oracle.

Where floating point decides the rank, both sides decide it in FP64 from
sums taken in descending order; their totals (the GPU's Gram trace, the
oracle's sum of all squared singular values) agree to rounding.  A rank that
differs is accepted only as a tie: the energy ratio at the boundary must then
be within 1e-9 of xi.  Store parity is block by block; query parity runs the
oracle's query phase on the downloaded store (decoupled, as in FP64 mode)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1805_00754_amd import synth
from paper_1805_00754_amd import zoomsvd as zs
from tests.gpu_common import (F32_KW, RANK_TOL_F32, TOL_FP32, TOL_FP64, compare_svd,
                              download_store, say, to_dev)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    zs.load()
    oracle.load()


def is_tie(s, k_a, k_b, xi):
    """Ranks k_a != k_b both within rounding of the rule for spectrum s."""
    s2 = np.sort(np.asarray(s, float) ** 2)[::-1]
    cum = np.cumsum(s2) / s2.sum()
    lo = min(k_a, k_b)
    return abs(k_a - k_b) == 1 and abs(cum[lo - 1] - xi) < 1e-9


CASES = [
    # name, t, c, b, k, dtype, mode, xi
    ("sinmix64_f64_xi90", 10_000, 64, 100, 10, torch.float64, zs.ZS_MODE_FP64, 0.90),
    ("sinmix64_f64_xi98", 10_000, 64, 100, 10, torch.float64, zs.ZS_MODE_FP64, 0.98),
    ("ar1_128_f64_xi95", 12_000, 128, 1_000, 20, torch.float64, zs.ZS_MODE_FP64, 0.95),
    ("sinmix48_f32_xi97", 6_000, 48, 250, 12, torch.float32, zs.ZS_MODE_FP32, 0.97),
]


def series(name, t, c, dtype):
    if name.startswith("ar1"):
        ser = synth.sinusoid_mixture(t, c, sources=12, seed=77, noise="ar1", noise_sigma=0.05)
    else:
        ser = synth.sinusoid_mixture(t, c, sources=8, seed=71 + c, noise="iid", noise_sigma=0.1,
                                     dtype="f32" if dtype == torch.float32 else "f64")
    return ser.A


@pytest.mark.parametrize("name,t,c,b,k,dtype,mode,xi", CASES)
def test_xi_store_and_queries(name, t, c, b, k, dtype, mode, xi):
    A = series(name, t, c, dtype)
    f32 = mode != zs.ZS_MODE_FP64
    tol, kw = (TOL_FP32, F32_KW) if f32 else (TOL_FP64, {})
    rank_tol = RANK_TOL_F32 if f32 else oracle.RANK_TOL
    say("xi", name)
    st = zs.zs_store_blocks(to_dev(A, dtype), b, k, mode=mode, xi=xi)
    zs.zs_sync_status(st)
    U, S, V, kk = download_store(st)
    ost = oracle.store(A, b, k, rank_tol=rank_tol, xi=xi)
    say("xi", name, "ranks kept:", np.bincount(ost.k_i, minlength=k + 1).tolist())
    ties = 0
    for i in range(st.nb):
        r = st.block_rows(i)
        if kk[i] != ost.k_i[i]:
            assert is_tie(np.linalg.svd(A[i * b:i * b + r], compute_uv=False), int(kk[i]),
                          int(ost.k_i[i]), xi), "block %d: k_i %d vs %d" % (i, kk[i], ost.k_i[i])
            ties += 1
            continue
        compare_svd((U[i * b:i * b + r], S[i], V[i], int(kk[i])),
                    (ost.U[i * b:i * b + r], ost.S[i], ost.V[i], int(ost.k_i[i])),
                    tol, c, "%s block %d" % (name, i), **kw)
    gst = oracle.store_from_arrays(st.t, st.c, st.b, st.k, U, S, V, kk, rank_tol=rank_tol, xi=xi)
    rng = synth.rng_for(400 + c)
    ts, te = synth.queries_uniform(rng, t, 8, 2, t)
    for q in range(len(ts)):
        kq = [k, max(1, k // 2)][q % 2]
        Ug, Sg, Vg, kg = zs.zs_query(st, int(ts[q]), int(te[q]), kq)
        zs.zs_sync_status(st)
        got = (Ug.double().cpu().numpy(), Sg.cpu().numpy(), Vg.double().cpu().numpy(), int(kg.item()))
        ref = oracle.query(gst, int(ts[q]), int(te[q]), kq)
        what = "%s query [%d,%d) kq %d" % (name, ts[q], te[q], kq)
        if got[3] != ref[3]:
            # a tie: moving xi by 1e-9 either way must reproduce the GPU's rank
            alt = [oracle.query(oracle.store_from_arrays(st.t, st.c, st.b, st.k, U, S, V, kk,
                                                         rank_tol=rank_tol, xi=xi + d),
                                int(ts[q]), int(te[q]), kq)[3] for d in (-1e-9, 1e-9)]
            assert got[3] in alt, "%s: k_out %d vs %d" % (what, got[3], ref[3])
            ties += 1
            continue
        compare_svd(got, ref, tol, c, what, **kw)
    assert ties <= 1, "%d rank ties: the rule's decisions disagree too often" % ties
    st.free()


def test_xi_batch_equals_single_and_off_equals_plain():
    ser = synth.sinusoid_mixture(8_000, 64, sources=8, seed=5, noise="iid", noise_sigma=0.1)
    A = to_dev(ser.A)
    st = zs.zs_store_blocks(A, 200, 12, xi=0.93)
    rng = synth.rng_for(33)
    ts, te = synth.queries_uniform(rng, 8_000, 20, 50, 7_000)
    kq = rng.integers(1, 13, size=20).astype(np.int32)
    batch = zs.zs_query_batch(st, ts, te, kq)
    torch.cuda.synchronize()
    for q in range(len(ts)):
        Ub, Sb, Vb, kb = [x.cpu() for x in batch.result(q)]
        Us, Ss, Vs, ks = [x.cpu() for x in zs.zs_query(st, int(ts[q]), int(te[q]), int(kq[q]))]
        assert int(kb[0]) == int(ks[0])
        assert torch.equal(Ub, Us) and torch.equal(Vb, Vs) and torch.equal(Sb, Ss)
    st.free()
    # xi = 1 turns the rule off: the plain store, bit for bit
    plain = zs.zs_store_blocks(A, 200, 12)
    off = zs.zs_store_blocks(A, 200, 12, xi=1.0)
    torch.cuda.synchronize()
    for x, y in zip(download_store(plain), download_store(off)):
        np.testing.assert_array_equal(x, y)
    a = [x.cpu() for x in zs.zs_query(plain, 77, 7_777, 12)]
    b = [x.cpu() for x in zs.zs_query(off, 77, 7_777, 12)]
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    plain.free()
    off.free()
