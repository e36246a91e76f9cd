"""Shared helpers of the GPU tests (parity of the HIP path against the oracle)."""
from __future__ import annotations

import sys

import numpy as np
import torch

from paper_1805_00754_amd import zoomsvd as zs
from tests.helpers import check_sigma, joint_sign_errs, orth_err, subspace_errs

# Tolerances of the FP64 path: relative error on sigma_1..k, switching to
# |error| / sigma_1 below 10 sqrt(c) u sigma_1; singular subspaces within
# TOL / g_j where g_j = (sigma_j - sigma_{j+1}) / sigma_1.
TOL_FP64 = 1e-10
# FP32 mode: block Gram on FP32 matrix cores, factors stored in FP32 (unit
# roundoff 6e-8); same rules.
TOL_FP32 = 1e-5
# BF16 mode: block Gram on BF16 matrix cores with FP32 accumulation; the input
# is rounded to bf16 (unit roundoff 3.9e-3) when it is wider.
TOL_BF16 = 1e-3
RANK_TOL_F32 = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(A: np.ndarray, dtype=None) -> torch.Tensor:
    t = torch.from_numpy(np.ascontiguousarray(A))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


F32_KW = dict(unit=6e-8, orth_v=1e-6, orth_u=1e-6)
# BF16 mode on input wider than bf16: the rounding of A is the unit roundoff
BF16_ROUND_KW = dict(unit=3.9e-3, orth_v=1e-6, orth_u=1e-6)


def mode_tol(mode: int) -> float:
    """Parity tolerance of a storage mode (relative error on sigma; subspaces
    within tol / gap)."""
    return {zs.ZS_MODE_FP64: TOL_FP64, zs.ZS_MODE_FP32: TOL_FP32, zs.ZS_MODE_BF16: TOL_BF16}[mode]


def download_store(st: zs.Store):
    """All block factors of a GPU store, in the oracle's layout (FP64; an FP32
    store's factors are widened exactly)."""
    U = np.zeros((st.t, st.k))
    S = np.zeros((st.nb, st.k))
    V = np.zeros((st.nb, st.c, st.k))
    kk = np.zeros(st.nb, np.int32)
    for i in range(st.nb):
        Ui, Si, Vi, ki = zs.zs_store_get_block(st, i)
        torch.cuda.synchronize()
        r = st.block_rows(i)
        U[i * st.b:i * st.b + r] = Ui.double().cpu().numpy()
        S[i] = Si.cpu().numpy()
        V[i] = Vi.double().cpu().numpy()
        kk[i] = int(ki.item())
    return U, S, V, kk


def compare_svd(got, ref, tol, c, what="", unit=1.1e-16, orth_v=1e-12, orth_u=1e-11):
    """got/ref = (U, s, V, k_out).  Asserts sigma, orthonormality, subspaces,
    the sign rule on V and the joint sign of each pair (u_j, v_j).  `unit` is
    the unit roundoff of the stored factors (switch to |error| / sigma_1 below
    10 sqrt(c) unit sigma_1).  With got's U = None only sigma, V and k_out are
    compared (the left factor of a very tall range is checked on a sample)."""
    Ug, sg, Vg, kg = got
    Ur, sr, Vr, kr = ref
    assert kg == kr, "%s: k_out %d vs %d" % (what, kg, kr)
    floor = 10.0 * np.sqrt(c) * unit
    e = check_sigma(sg, sr, tol, floor)
    if e > 1.0:
        say("%s: sigma got %s" % (what, np.array2string(np.asarray(sg), precision=12)))
        say("%s: sigma ref %s" % (what, np.array2string(np.asarray(sr), precision=12)))
    assert e <= 1.0, "%s: sigma error %.3g x tol" % (what, e)
    assert np.all(sg[kg:] == 0), what
    assert np.all(Vg[:, kg:] == 0), what
    assert orth_err(Vg[:, :kg]) < orth_v, what
    ev = subspace_errs(Vg[:, :kg], Vr[:, :kg], sr[:kg], tol)
    assert ev <= 1.0, "%s: subspace error V %.3g (x tol/gap)" % (what, ev)
    # sign rule: largest-|v| entry positive
    for j in range(kg):
        assert Vg[np.argmax(np.abs(Vg[:, j])), j] > 0, what
    if Ug is None:
        return e, ev, None
    assert np.all(Ug[:, kg:] == 0), what
    assert orth_err(Ug[:, :kg]) < orth_u, what
    eu = subspace_errs(Ug[:, :kg], Ur[:, :kg], sr[:kg], tol)
    assert eu <= 1.0, "%s: subspace error U %.3g (x tol/gap)" % (what, eu)
    nbad = joint_sign_errs(Ug[:, :kg], Vg[:, :kg], Ur[:, :kg], Vr[:, :kg], sr[:kg], tol)
    assert nbad == 0, "%s: %d pairs (u_j, v_j) with a sign flipped against the oracle's" % (what, nbad)
    return e, ev, eu
