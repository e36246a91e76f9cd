"""Pins for the oracle's SVD primitive (Sec. 2.1): closed forms, an
independent library (LAPACK through numpy), invariants, Eckart-Young."""
import numpy as np
import pytest

from tests.helpers import orth_err, sin_theta


def test_1x1(orc):
    U, s, V, rank, _ = orc.svd(np.array([[-3.5]]))
    assert rank == 1
    assert s[0] == 3.5
    assert U[0, 0] * s[0] * V[0, 0] == -3.5
    assert V[0, 0] == 1.0          # sign rule: largest |v| entry positive


@pytest.mark.parametrize("abcd", [(1.0, 2.0, 3.0, 4.0), (2.0, -1.0, 0.5, 3.0), (0.0, 1.0, -1.0, 0.0),
                                  (5.0, 0.0, 0.0, 1e-3)])
def test_2x2_closed_form(orc, abcd):
    # sigma_1 + sigma_2 = sqrt((a+d)^2 + (b-c)^2), sigma_1 - sigma_2 = sqrt((a-d)^2 + (b+c)^2)
    a, b, c, d = abcd
    p = np.hypot(a + d, b - c)
    q = np.hypot(a - d, b + c)
    U, s, V, _, _ = orc.svd(np.array([[a, b], [c, d]]))
    np.testing.assert_allclose(s, [(p + q) / 2, abs(p - q) / 2], rtol=1e-14, atol=1e-15)


def test_diagonal(orc):
    d = np.array([0.5, -7.0, 3.0, 0.0, 2.0])
    U, s, V, rank, _ = orc.svd(np.diag(d))
    np.testing.assert_array_equal(s, [7.0, 3.0, 2.0, 0.5, 0.0])
    assert rank == 4
    # singular vectors are signed unit vectors
    for j, idx in enumerate([1, 2, 4, 0]):
        assert abs(abs(V[idx, j]) - 1.0) < 1e-15


def test_orthogonal_has_unit_singular_values(orc):
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    _, s, _, rank, _ = orc.svd(Q)
    assert rank == 40
    np.testing.assert_allclose(s, np.ones(40), atol=2e-14)


def test_rank_one(orc):
    rng = np.random.default_rng(2)
    x = rng.standard_normal(30)
    y = rng.standard_normal(7)
    U, s, V, rank, _ = orc.svd(np.outer(x, y))
    assert rank == 1
    np.testing.assert_allclose(s[0], np.linalg.norm(x) * np.linalg.norm(y), rtol=1e-14)
    assert np.all(s[1:] == 0)
    assert sin_theta(U[:, :1], x[:, None]) < 1e-14
    assert sin_theta(V[:, :1], y[:, None]) < 1e-14


@pytest.mark.parametrize("shape", [(3, 3), (10, 4), (4, 10), (100, 64), (64, 100), (257, 31), (1, 9), (9, 1)])
def test_against_lapack(orc, shape):
    rng = np.random.default_rng(sum(shape))
    A = rng.standard_normal(shape)
    U, s, V, rank, sweeps = orc.svd(A)
    ref = np.linalg.svd(A, compute_uv=True, full_matrices=False)
    Ur, sr, Vrt = ref
    assert sweeps > 0
    assert rank == min(shape)
    np.testing.assert_allclose(s, sr, rtol=1e-13)
    # singular vectors (sign-invariant) where the gaps are healthy
    for j in range(len(s)):
        gap = min([abs(sr[j] - sr[i]) for i in range(len(sr)) if i != j] or [1.0]) / sr[0]
        if gap > 1e-6:
            assert abs(abs(U[:, j] @ Ur[:, j]) - 1) < 1e-12 / gap
            assert abs(abs(V[:, j] @ Vrt[j]) - 1) < 1e-12 / gap


@pytest.mark.parametrize("shape", [(200, 20), (20, 200), (64, 64)])
def test_invariants(orc, shape):
    rng = np.random.default_rng(7)
    A = rng.standard_normal(shape) @ np.diag(np.logspace(0, -6, shape[1]))
    U, s, V, rank, _ = orc.svd(A)
    assert orth_err(U) < 1e-13 * max(shape)
    assert orth_err(V) < 1e-13 * max(shape)
    assert np.linalg.norm(A @ V - U * s) <= 1e-14 * max(shape) * np.linalg.norm(A)
    assert np.all(np.diff(s) <= 0)
    # sign rule: the largest-magnitude entry of every v_j is positive
    for j in range(rank):
        assert V[np.argmax(np.abs(V[:, j])), j] > 0


@pytest.mark.parametrize("k", [1, 3, 8])
def test_eckart_young(orc, k):
    rng = np.random.default_rng(k)
    A = rng.standard_normal((50, 12))
    U, s, V, _, _ = orc.svd(A)
    Ak = (U[:, :k] * s[:k]) @ V[:, :k].T
    err = np.linalg.norm(A - Ak) ** 2
    np.testing.assert_allclose(err, np.sum(s[k:] ** 2), rtol=1e-12)


def test_rank_deficient_and_zero(orc):
    rng = np.random.default_rng(3)
    A = rng.standard_normal((60, 4)) @ rng.standard_normal((4, 15))
    U, s, V, rank, _ = orc.svd(A)
    assert rank == 4
    assert np.all(s[4:] == 0)
    assert np.all(U[:, 4:] == 0) and np.all(V[:, 4:] == 0)
    sr = np.linalg.svd(A, compute_uv=False)
    np.testing.assert_allclose(s[:4], sr[:4], rtol=1e-13)
    U, s, V, rank, _ = orc.svd(np.zeros((5, 3)))
    assert rank == 0 and np.all(s == 0) and np.all(U == 0) and np.all(V == 0)


def test_nvec_limits_vectors_only(orc):
    rng = np.random.default_rng(4)
    A = rng.standard_normal((80, 10))
    U, s, V, rank, _ = orc.svd(A, nvec=3)
    Uf, sf, Vf, _, _ = orc.svd(A)
    np.testing.assert_array_equal(s, sf)
    np.testing.assert_array_equal(U[:, :3], Uf[:, :3])
    assert np.all(U[:, 3:] == 0) and np.all(V[:, 3:] == 0)
    assert rank == 10
