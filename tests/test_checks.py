"""The comparison rules of the GPU parity tests, checked on the CPU: each
accepts a correct SVD under the freedoms the SVD has (a joint sign per pair,
rotations inside a repeated singular value) and rejects planted mistakes."""
import numpy as np

from tests.gpu_common import compare_svd
from tests.helpers import joint_sign_errs

import pytest


def _svd(m, n, k, seed, spectrum=None):
    rng = np.random.default_rng(seed)
    Q1, _ = np.linalg.qr(rng.standard_normal((m, k)))
    Q2, _ = np.linalg.qr(rng.standard_normal((n, k)))
    s = np.sort(rng.uniform(1.0, 10.0, k))[::-1] if spectrum is None else np.asarray(spectrum, float)
    for j in range(k):           # sign rule of the library: largest |v| entry positive
        if Q2[np.argmax(np.abs(Q2[:, j])), j] < 0:
            Q2[:, j] *= -1
            Q1[:, j] *= -1
    return Q1, s, Q2


def test_joint_sign_accepts_pairs_flipped_together():
    U, s, V = _svd(200, 30, 6, 1)
    U2, V2 = U.copy(), V.copy()
    U2[:, 2] *= -1
    V2[:, 2] *= -1
    assert joint_sign_errs(U2, V2, U, V, s, 1e-10) == 0


def test_joint_sign_catches_one_flipped_vector():
    U, s, V = _svd(200, 30, 6, 2)
    for j in range(6):
        U2 = U.copy()
        U2[:, j] *= -1           # U Sigma V^T changes: u_j flipped against v_j
        assert joint_sign_errs(U2, V, U, V, s, 1e-10) == 1


def test_compare_svd_catches_flip_but_not_rotation_in_a_tie():
    U, s, V = _svd(300, 20, 5, 3, spectrum=[9.0, 5.0, 5.0, 2.0, 1.0])
    kk = 5
    ref = (U, s, V, kk)
    # a rotation inside the repeated value 5 applied to both factors is a valid SVD
    th = 0.3
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    U2, V2 = U.copy(), V.copy()
    U2[:, 1:3] = U[:, 1:3] @ R
    V2[:, 1:3] = V[:, 1:3] @ R
    for j in (1, 2):
        if V2[np.argmax(np.abs(V2[:, j])), j] < 0:
            V2[:, j] *= -1
            U2[:, j] *= -1
    compare_svd((U2, s.copy(), V2, kk), ref, 1e-10, 20, "rotated tie")
    # u_0 flipped alone: rejected
    U3 = U.copy()
    U3[:, 0] *= -1
    with pytest.raises(AssertionError, match="sign flipped"):
        compare_svd((U3, s.copy(), V, kk), ref, 1e-10, 20, "flip")
    # U not given: sigma and V still compared
    compare_svd((None, s.copy(), V, kk), ref, 1e-10, 20, "no U")
    s4 = s.copy()
    s4[3] *= 1 + 1e-8
    with pytest.raises(AssertionError, match="sigma"):
        compare_svd((None, s4, V, kk), ref, 1e-10, 20, "sigma")
