"""FP32 and BF16 modes: the block Gram runs on the FP32 or BF16 matrix cores
(FP32 accumulation), the eigen-solves and the refinement (projection and
Rayleigh-Ritz) in FP64; the store keeps U and V in FP32 and answers in FP32.
Tolerances: 1e-5 (FP32 mode) and 1e-3 (BF16 mode).

Input is exactly representable in the mode's input type (synthetic data
rounded to float32 or bfloat16), so the oracle sees the same values in FP64;
one case feeds float32 input to BF16 mode, which rounds it to bf16 for the
Gram.  Store parity is block by block; query parity runs the oracle's query
phase on the store downloaded from the GPU (decoupled, as in FP64 mode)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1805_00754_amd import synth
from paper_1805_00754_amd import zoomsvd as zs
from tests.gpu_common import (BF16_ROUND_KW, F32_KW, RANK_TOL_F32, compare_svd, download_store,
                              mode_tol, say, to_dev)

pytestmark = pytest.mark.gpu

MODES = [("f32", torch.float32, zs.ZS_MODE_FP32), ("bf16", torch.bfloat16, zs.ZS_MODE_BF16)]


@pytest.fixture(scope="module", autouse=True)
def _lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    zs.load()
    oracle.load()


def series(dtype_name, t, c, seed):
    ser = synth.sinusoid_mixture(t, c, sources=min(6, c), seed=seed, noise="iid",
                                 noise_sigma=0.1, dtype=dtype_name)
    return ser.A          # float64 array of values exact in the input type


@pytest.mark.parametrize("name,tdtype,mode", MODES)
@pytest.mark.parametrize("t,c,b,k", [(4_000, 64, 250, 10), (3_100, 128, 1000, 20), (900, 33, 64, 33),
                                     (4_000, 256, 1000, 32)])
def test_store_and_query_parity(name, tdtype, mode, t, c, b, k):
    A = series(name, t, c, seed=11 + c)
    say("precision", name, (t, c, b, k))
    st = zs.zs_store_blocks(to_dev(A, tdtype), b, k, mode=mode)
    torch.cuda.synchronize()
    assert st.out_dtype == torch.float32
    U, S, V, kk = download_store(st)
    ost = oracle.store(A, b, k, rank_tol=RANK_TOL_F32)
    tol = mode_tol(mode)
    for i in range(st.nb):
        r = st.block_rows(i)
        compare_svd((U[i * b:i * b + r], S[i], V[i], int(kk[i])),
                    (ost.U[i * b:i * b + r], ost.S[i], ost.V[i], int(ost.k_i[i])),
                    tol, c, "%s store block %d" % (name, i), **F32_KW)
    gst = oracle.store_from_arrays(st.t, st.c, st.b, st.k, U, S, V, kk, rank_tol=RANK_TOL_F32)
    rng = synth.rng_for(90 + c)
    ts, te = synth.queries_uniform(rng, t, 6, 1, t)
    for q in range(len(ts)):
        kq = [k, 1, max(1, k // 2)][q % 3]
        Ug, Sg, Vg, kg = zs.zs_query(st, int(ts[q]), int(te[q]), kq)
        zs.zs_sync_status(st)
        assert Ug.dtype == torch.float32 and Vg.dtype == torch.float32 and Sg.dtype == torch.float64
        got = (Ug.double().cpu().numpy(), Sg.cpu().numpy(), Vg.double().cpu().numpy(), int(kg.item()))
        ref = oracle.query(gst, int(ts[q]), int(te[q]), kq)
        compare_svd(got, ref, tol, c, "%s query [%d,%d) kq %d" % (name, ts[q], te[q], kq),
                    **F32_KW)
    st.free()


@pytest.mark.parametrize("name,tdtype,mode", MODES)
def test_batch_equals_single_bitwise(name, tdtype, mode):
    A = series(name, 5_000, 48, seed=3)
    st = zs.zs_store_blocks(to_dev(A, tdtype), 200, 12, mode=mode)
    rng = synth.rng_for(5)
    ts, te = synth.queries_uniform(rng, 5_000, 24, 100, 4_000)
    kq = rng.integers(1, 13, size=24).astype(np.int32)
    batch = zs.zs_query_batch(st, ts, te, kq)
    torch.cuda.synchronize()
    for q in range(len(ts)):
        Ub, Sb, Vb, kb = [x.cpu() for x in batch.result(q)]
        Us, Ss, Vs, ks = [x.cpu() for x in zs.zs_query(st, int(ts[q]), int(te[q]), int(kq[q]))]
        assert int(kb[0]) == int(ks[0])
        assert torch.equal(Ub, Us) and torch.equal(Vb, Vs) and torch.equal(Sb, Ss)
    st.free()


def test_fp64_mode_accepts_float32_input():
    """FP64 mode reads FP32 input and widens it exactly: same store as FP64 input."""
    A = series("f32", 2_000, 32, seed=8)
    st32 = zs.zs_store_blocks(to_dev(A, torch.float32), 250, 8, mode=zs.ZS_MODE_FP64)
    st64 = zs.zs_store_blocks(to_dev(A), 250, 8, mode=zs.ZS_MODE_FP64)
    a, b = download_store(st32), download_store(st64)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


# The wide workload's geometry (c = 1024, k = 64, b = 4096, bf16-valued input
# with singular values decaying as 0.9^j, a 1,152-row last block) at a reduced
# t of two full blocks plus the tail.  The same values go in as bfloat16 (BF16
# mode) and as float32 (FP32 mode), so one oracle store serves both.
WIDE_T = 2 * 4096 + 1152


@pytest.fixture(scope="module")
def wide():
    ser, cfg = synth.workload("decay_2m_x1024_bf16", t=WIDE_T)
    say("wide: oracle store", ser.A.shape)
    ost = oracle.store(ser.A, cfg["b"], cfg["k"], rank_tol=RANK_TOL_F32)
    return ser, cfg, ost


@pytest.mark.parametrize("name,tdtype,mode", [("bf16", torch.bfloat16, zs.ZS_MODE_BF16),
                                              ("f32", torch.float32, zs.ZS_MODE_FP32)])
def test_wide_geometry_parity(wide, name, tdtype, mode):
    ser, cfg, ost = wide
    A = ser.A
    b, k = cfg["b"], cfg["k"]
    c = A.shape[1]
    say("wide", name, A.shape, b, k)
    st = zs.zs_store_blocks(to_dev(A, tdtype), b, k, mode=mode)
    torch.cuda.synchronize()
    assert st.nb == 3 and st.block_rows(2) == 1152
    U, S, V, kk = download_store(st)
    tol = mode_tol(mode)
    for i in range(st.nb):
        r = st.block_rows(i)
        compare_svd((U[i * b:i * b + r], S[i], V[i], int(kk[i])),
                    (ost.U[i * b:i * b + r], ost.S[i], ost.V[i], int(ost.k_i[i])),
                    tol, c, "wide %s block %d" % (name, i), **F32_KW)
    gst = oracle.store_from_arrays(st.t, st.c, st.b, st.k, U, S, V, kk, rank_tol=RANK_TOL_F32)
    # ranges over the tail, across both block edges, inside one block, and all rows
    for ts, te, kq in [(0, WIDE_T, k), (1_000, 9_000, k), (4_000, 4_200, 16), (8_200, WIDE_T, 32),
                       (3_000, 8_500, 8)]:
        Ug, Sg, Vg, kg = zs.zs_query(st, ts, te, kq)
        zs.zs_sync_status(st)
        got = (Ug.double().cpu().numpy(), Sg.cpu().numpy(), Vg.double().cpu().numpy(), int(kg.item()))
        ref = oracle.query(gst, ts, te, kq)
        compare_svd(got, ref, tol, c, "wide %s [%d,%d) kq %d" % (name, ts, te, kq), **F32_KW)
    st.free()


def test_bf16_mode_rounds_wider_input():
    """float32 input in BF16 mode (the 4M x 256 workload's geometry at reduced
    t, with a short last block): the Gram sees A rounded to bf16, the
    refinement the float32 values; parity at the BF16 tolerance against the
    oracle on the float32 values."""
    ser, cfg = synth.workload("sinmix_4m_x256_f32", t=2 * 2000 + 700)
    A, b, k = ser.A, cfg["b"], cfg["k"]
    c = A.shape[1]
    st = zs.zs_store_blocks(to_dev(A, torch.float32), b, k, mode=zs.ZS_MODE_BF16)
    torch.cuda.synchronize()
    assert st.nb == 3 and st.block_rows(2) == 700
    U, S, V, kk = download_store(st)
    ost = oracle.store(A, b, k, rank_tol=RANK_TOL_F32)
    tol = mode_tol(zs.ZS_MODE_BF16)
    for i in range(st.nb):
        r = st.block_rows(i)
        compare_svd((U[i * b:i * b + r], S[i], V[i], int(kk[i])),
                    (ost.U[i * b:i * b + r], ost.S[i], ost.V[i], int(ost.k_i[i])),
                    tol, c, "bf16-rounded block %d" % i, **BF16_ROUND_KW)
    gst = oracle.store_from_arrays(st.t, st.c, st.b, st.k, U, S, V, kk, rank_tol=RANK_TOL_F32)
    for ts, te, kq in [(0, st.t, k), (1_500, 4_400, 16), (100, 1_900, 8)]:
        Ug, Sg, Vg, kg = zs.zs_query(st, ts, te, kq)
        zs.zs_sync_status(st)
        got = (Ug.double().cpu().numpy(), Sg.cpu().numpy(), Vg.double().cpu().numpy(), int(kg.item()))
        compare_svd(got, oracle.query(gst, ts, te, kq), tol, c, "bf16-rounded [%d,%d)" % (ts, te),
                    **F32_KW)
    st.free()
