"""GPU tests of zs_query_noalloc, the query entry point that allocates nothing
(its scratch is a fixed device array shared by every such call on the GPU).

Each case makes two calls in a row on one store, the second with a smaller
range, and checks every output against zs_query on the same range bit for
bit (both run the same kernels on the same inputs) and against the oracle's
query phase on the store downloaded from the GPU (Alg. 2 with Alg. 3).
"""
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


def run(st, ts, te, kq, noalloc, ld_pad=0):
    n = te - ts
    dev = torch.device("cuda", 0)
    U = torch.full((n, kq + ld_pad), 7.0, dtype=st.out_dtype, device=dev)
    V = torch.full((st.c, kq + ld_pad), 7.0, dtype=st.out_dtype, device=dev)
    S = torch.full((kq,), 7.0, dtype=torch.float64, device=dev)
    ko = torch.full((1,), -1, dtype=torch.int32, device=dev)
    zs.zs_query(st, ts, te, kq, U=U, S=S, V=V, k_out=ko, noalloc=noalloc)
    zs.zs_sync_status(st)
    return U.cpu(), S.cpu(), V.cpu(), int(ko.item())


CASES = [
    # (t, c, b, k, mode, [(t_s, t_e, k_q, ld_pad), second call smaller])
    (21_100, 128, 1000, 20, zs.ZS_MODE_FP64, [(437, 20_960, 20, 0), (3_010, 3_777, 12, 3)]),
    (6_200, 256, 1000, 32, zs.ZS_MODE_FP64, [(123, 6_200, 32, 0), (2_000, 3_000, 16, 0)]),
    (9_000, 64, 250, 10, zs.ZS_MODE_FP32, [(0, 8_999, 10, 2), (501, 502, 3, 0)]),
]


@pytest.mark.parametrize("t,c,b,k,mode,calls", CASES)
def test_noalloc_equals_query(t, c, b, k, mode, calls):
    ser = synth.sinusoid_mixture(t, c, sources=min(12, c), seed=31 + c, noise="iid",
                                 noise_sigma=0.1)
    st = zs.zs_store_blocks(to_dev(ser.A), b, k, mode=mode)
    torch.cuda.synchronize()
    Ug, Sg, Vg, kg = download_store(st)
    f64 = mode == zs.ZS_MODE_FP64
    ost = oracle.store_from_arrays(t, c, b, k, Ug, Sg, Vg, kg,
                                   **({} if f64 else dict(rank_tol=RANK_TOL_F32)))
    tol, kw = (TOL_FP64, {}) if f64 else (TOL_FP32, F32_KW)
    for ts, te, kq, pad in calls:
        say("noalloc c=%d mode=%d [%d, %d) k_q=%d pad=%d" % (c, mode, ts, te, kq, pad))
        a = run(st, ts, te, kq, True, pad)
        r = run(st, ts, te, kq, False, pad)
        assert a[3] == r[3]
        for x, y in zip(a[:3], r[:3]):
            assert torch.equal(x, y), "zs_query_noalloc differs from zs_query"
        got = (a[0][:, :kq].double().numpy(), a[1].numpy(), a[2][:, :kq].double().numpy(), a[3])
        ref = oracle.query(ost, ts, te, kq)
        compare_svd(got, ref, tol, c, "noalloc [%d, %d)" % (ts, te), **kw)
        if pad:                          # columns past k_q of a strided output are untouched
            assert torch.all(a[0][:, kq:] == 7.0) and torch.all(a[2][:, kq:] == 7.0)
    st.free()


def test_noalloc_rejects_query_beyond_scratch():
    # 10,000 blocks of 32 rows at k = k_q = 32: Y and C alone need 2 x 82 MB
    t, c, b, k = 320_000, 64, 32, 32
    ser = synth.sinusoid_mixture(t, c, sources=8, seed=5, noise="iid", noise_sigma=0.1)
    st = zs.zs_store_blocks(to_dev(ser.A), b, k)
    torch.cuda.synchronize()
    with pytest.raises(zs.ZSError) as ei:
        run(st, 0, t, k, True)
    assert ei.value.status == zs.ZS_ENOMEM
    assert "scratch" in zs.zs_last_error()
    # a range that fits still runs, and matches zs_query bit for bit
    a = run(st, 1_000, 41_017, 16, True)
    r = run(st, 1_000, 41_017, 16, False)
    assert a[3] == r[3] and all(torch.equal(x, y) for x, y in zip(a[:3], r[:3]))
    st.free()
