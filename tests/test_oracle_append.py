"""Pins for the oracle's streaming ingest (Alg. 1's incremental update,
Eqs. (2)-(3), for appended rows at once).  The update is exact: with every
block of rank <= k, or with k = c, a store grown by appends reconstructs the
data like the store of all rows at once and has the same block spectra, for a
last block that is partial, full, or filled and overflowed by the append."""
import numpy as np
import pytest

from paper_1805_00754_amd import synth


def check_same(a, b, A):
    assert a.t == b.t and a.nb == b.nb
    np.testing.assert_array_equal(a.k_i, b.k_i)
    assert np.allclose(a.S, b.S, rtol=1e-11, atol=1e-12 * np.abs(b.S).max())
    for i in range(a.nb):
        r = a.block_rows(i)
        Ai = (a.U[i * a.b:i * a.b + r] * a.S[i]) @ a.V[i].T
        assert np.allclose(Ai, A[i * a.b:i * a.b + r], atol=1e-9 * np.abs(A).max()), i


@pytest.mark.parametrize("t0,cuts", [(430, [37, 200, 333]), (500, [100]), (57, [43]), (10, [1, 1, 500])])
def test_appends_equal_batch_on_block_rank_le_k(orc, t0, cuts):
    # every 100-row block has rank 3 <= k, so the partial last blocks do too
    A = synth.block_low_rank(1_100, 8, 100, rank=3, seed=12)
    st = orc.store(A[:t0], 100, 5)
    pos = t0
    for m in cuts:
        st = orc.append(st, A[pos:pos + m])
        pos += m
    ref = orc.store(A[:pos], 100, 5)
    check_same(st, ref, A[:pos])


def test_append_with_k_equal_c_is_exact_on_noisy_data(orc):
    ser = synth.sinusoid_mixture(900, 6, sources=3, seed=2, noise="iid", noise_sigma=0.2)
    A = ser.A
    st = orc.store(A[:250], 120, 6)
    st = orc.append(st, A[250:610])
    ref = orc.store(A[:610], 120, 6)
    check_same(st, ref, A[:610])


def test_queries_after_append_match_direct(orc):
    A = synth.block_low_rank(1_000, 9, 50, rank=3, seed=31)
    st = orc.append(orc.store(A[:333], 50, 9), A[333:1_000])
    for ts, te in [(0, 1_000), (310, 777), (330, 340), (512, 999)]:
        U, s, V, ko = orc.query(st, ts, te, 9)
        Ud, sd, Vd, kd = orc.direct(A, ts, te, 9)
        assert ko == kd
        assert np.allclose(s, sd, rtol=1e-10, atol=1e-12)
        assert np.allclose((U * s) @ V.T, A[ts:te], atol=1e-9)


def test_append_truncation_is_never_better_than_optimal(orc):
    """With truncation the grown last block is a rank-k approximation of its
    rows, so by Eckart-Young its error is at least the optimal one."""
    ser = synth.sinusoid_mixture(700, 10, sources=6, seed=8, noise="iid", noise_sigma=0.3)
    A = ser.A
    st = orc.append(orc.store(A[:230], 300, 3), A[230:300])
    blk = A[:300]
    Ai = (st.U[:300] * st.S[0]) @ st.V[0].T
    s = np.linalg.svd(blk, compute_uv=False)
    assert np.linalg.norm(blk - Ai) >= np.sqrt((s[3:] ** 2).sum()) * (1 - 1e-12)
