"""The first-stage eigen-solver has two launch forms: with more problems than
the device has CUs, 512-thread work-groups share a CU two at a time; with
fewer, 1,024-thread work-groups take a CU each.  Both sum in the same order,
so a problem's result does not depend on how many are solved with it.  Here a
batch of more queries than CUs is compared bit for bit with each query alone,
and a store of more blocks than CUs with the store of single blocks, for c in
each of the solver's size classes (c <= 32, <= 64, <= 128)."""
import numpy as np
import pytest
import torch

from paper_1805_00754_amd import synth
from paper_1805_00754_amd import zoomsvd as zs
from tests.gpu_common import download_store, say, to_dev

pytestmark = pytest.mark.gpu


def n_cus():
    return torch.cuda.get_device_properties(0).multi_processor_count


@pytest.fixture(scope="module", autouse=True)
def _lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    zs.load()


@pytest.mark.parametrize("c,k", [(128, 20), (48, 12), (24, 8)])
def test_batch_form_equals_single_form(c, k):
    t, b = 60_000, 400
    ser = synth.sinusoid_mixture(t, c, sources=8, seed=300 + c, noise="ar1", noise_sigma=0.05)
    st = zs.zs_store_blocks(to_dev(ser.A), b, k)
    nq = n_cus() + 13
    rng = synth.rng_for(900 + c)
    ts, te = synth.queries_uniform(rng, t, nq, 150, 30_000)
    kq = rng.integers(1, k + 1, size=nq).astype(np.int32)
    say("eig forms: batch of", nq, "queries, c", c)
    batch = zs.zs_query_batch(st, ts, te, kq)
    torch.cuda.synchronize()
    for q in range(nq):
        Ub, Sb, Vb, kb = [x.cpu() for x in batch.result(q)]
        Us, Ss, Vs, ks = [x.cpu() for x in zs.zs_query(st, int(ts[q]), int(te[q]), int(kq[q]))]
        what = "query %d [%d,%d) kq %d" % (q, ts[q], te[q], kq[q])
        assert int(kb[0]) == int(ks[0]), what
        assert torch.equal(Sb, Ss), what
        assert torch.equal(Vb, Vs), what
        assert torch.equal(Ub, Us), what
    st.free()


@pytest.mark.parametrize("c,k", [(128, 20), (40, 10)])
def test_store_form_equals_single_block_form(c, k):
    b = 200
    nb = n_cus() + 5
    t = nb * b - 77                                # a short last block
    ser = synth.sinusoid_mixture(t, c, sources=6, seed=500 + c, noise="iid", noise_sigma=0.1)
    say("eig forms: store of", nb, "blocks, c", c)
    st = zs.zs_store_blocks(to_dev(ser.A), b, k)
    torch.cuda.synchronize()
    U, S, V, kk = download_store(st)
    for i in (0, nb // 2, nb - 1):
        r = st.block_rows(i)
        one = zs.zs_store_blocks(to_dev(np.ascontiguousarray(ser.A[i * b:i * b + r])), b, k)
        torch.cuda.synchronize()
        U1, S1, V1, kk1 = download_store(one)
        what = "block %d" % i
        assert kk1[0] == kk[i], what
        np.testing.assert_array_equal(S1[0], S[i], err_msg=what)
        np.testing.assert_array_equal(V1[0], V[i], err_msg=what)
        np.testing.assert_array_equal(U1[:r], U[i * b:i * b + r], err_msg=what)
        one.free()
    st.free()
