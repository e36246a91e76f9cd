"""Comparison helpers shared by the tests (sign- and rotation-invariant)."""
from __future__ import annotations

import numpy as np


def orth_err(Q: np.ndarray) -> float:
    """max |Q^T Q - I| over the non-zero columns of Q."""
    if Q.size == 0:
        return 0.0
    keep = np.linalg.norm(Q, axis=0) > 0
    Q = Q[:, keep]
    return float(np.abs(Q.T @ Q - np.eye(Q.shape[1])).max()) if Q.shape[1] else 0.0


def sin_theta(A: np.ndarray, B: np.ndarray) -> float:
    """sin of the largest principal angle between span(A) and span(B)
    (both with orthonormal columns, same count)."""
    if A.shape[1] == 0:
        return 0.0
    qa, _ = np.linalg.qr(A)
    qb, _ = np.linalg.qr(B)
    # sin of the largest angle = || (I - Qa Qa^T) Qb ||_2 (accurate for small angles)
    resid = qb - qa @ (qa.T @ qb)
    return float(np.linalg.norm(resid, 2))


def check_sigma(s_hat, s_ref, rtol, abs_floor_rel, n_check=None):
    """Relative error on sigma_1..n, switching to error/sigma_1 below the
    floor abs_floor_rel * sigma_1.  Returns the worst normalised error."""
    s_hat = np.asarray(s_hat, float)
    s_ref = np.asarray(s_ref, float)
    n = len(s_ref) if n_check is None else n_check
    s1 = max(float(s_ref[0]), 1e-300) if len(s_ref) else 1.0
    worst = 0.0
    for j in range(n):
        d = abs(s_hat[j] - s_ref[j])
        if s_ref[j] > abs_floor_rel * s1:
            e = d / s_ref[j]
        else:
            e = d / s1
        worst = max(worst, e / rtol)
    return worst


def subspace_errs(U_hat, U_ref, s_ref, tol):
    """For every j with a relative gap g_j = (s_j - s_{j+1}) / s_1 >= 1e-8,
    sin theta(span U_hat[:, :j+1], span U_ref[:, :j+1]) must be <= tol / g_j.
    Returns the worst ratio (<= 1 passes)."""
    s_ref = np.asarray(s_ref, float)
    r = int((s_ref > 0).sum())
    if r == 0:
        return 0.0
    s1 = s_ref[0]
    worst = 0.0
    for j in range(r):
        nxt = s_ref[j + 1] if j + 1 < len(s_ref) else 0.0
        g = (s_ref[j] - nxt) / s1
        if g < 1e-8:
            continue
        st = sin_theta(U_hat[:, : j + 1], U_ref[:, : j + 1])
        worst = max(worst, st / (tol / g))
    return worst


def joint_sign_errs(U_hat, V_hat, U_ref, V_ref, s_ref, tol, min_angle=0.1):
    """The SVD fixes each pair (u_j, v_j) only up to a JOINT sign: flipping
    u_j alone changes U Sigma V^T (Sec. 2.1).  For every isolated j (relative
    gaps to both neighbours >= 1e-8, and tol / gap <= min_angle so that the
    subspace tests pin each vector to within that angle), the overlaps
    u_hat_j . u_j and v_hat_j . v_j must have the same sign.  Returns the
    number of pairs that violate it."""
    s_ref = np.asarray(s_ref, float)
    r = int((s_ref > 0).sum())
    if r == 0:
        return 0
    s1 = s_ref[0]
    bad = 0
    for j in range(r):
        nxt = s_ref[j + 1] if j + 1 < len(s_ref) else 0.0
        g = (s_ref[j] - nxt) / s1
        if j > 0:
            g = min(g, (s_ref[j - 1] - s_ref[j]) / s1)
        if g < 1e-8 or tol / g > min_angle:
            continue
        pu = float(U_hat[:, j] @ U_ref[:, j])
        pv = float(V_hat[:, j] @ V_ref[:, j])
        if not (pu * pv > 0.0):
            bad += 1
    return bad
