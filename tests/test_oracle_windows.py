"""Pins for the oracle's window similarity (the case study of Sec. 5): on data
of rank <= k in every block the stitched SVD of any range is its direct SVD,
so each window's u_1, and the cosines, must equal those from LAPACK's SVD of
the raw window; a window whose rows repeat the base gives cosine 1."""
import numpy as np

from paper_1805_00754_amd import synth


def lapack_u1(X):
    """u_1 of X with the sign rule (largest-|v_1| entry positive)."""
    U, s, Vt = np.linalg.svd(X, full_matrices=False)
    u, v = U[:, 0], Vt[0]
    return u if v[np.argmax(np.abs(v))] > 0 else -u


def periodic_low_rank(period, reps, c, rank, seed):
    rng = synth.rng_for(seed)
    L = rng.standard_normal((period, rank))
    R = rng.standard_normal((rank, c))
    one = L @ R
    return np.vstack([one] * reps)


def test_windows_match_lapack_on_exact_data(orc):
    A = periodic_low_rank(600, 5, 9, rank=3, seed=4)       # global rank 3 <= k
    st = orc.store(A, 70, 5)
    ts, te, stride, nw = 1_900, 2_420, 50, 30
    sim = orc.window_similarity(st, ts, te, stride, nw)
    u0 = lapack_u1(A[ts:te])
    for w in range(1, nw + 1):
        uw = lapack_u1(A[ts - w * stride:te - w * stride])
        assert abs(sim[w - 1] - u0 @ uw) < 1e-9, w
    # windows 12 and 24 (shifts of 600 = one period) repeat the base
    assert abs(sim[11] - 1.0) < 1e-12 and abs(sim[23] - 1.0) < 1e-12
    assert set(np.argsort(-sim)[:2]) == {11, 23}
