"""Pins for the oracle's energy-threshold rank (Eq. (1)): with 0 < xi < 1 every
low-rank approximation of the method keeps the smallest rank whose leading
squared singular values reach xi times the sum of all of them.

The pins use matrices built with prescribed singular values (hand-computed
expected ranks), LAPACK's SVD through numpy as an independent spectrum, and
exactly low-rank data on which the stitched SVD equals the direct one; planted
mistakes in the rule are caught."""
import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

from paper_1805_00754_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def prescribed(m, n, s, rng):
    """m x n matrix with singular values s (random singular vectors)."""
    r = len(s)
    Q1 = np.linalg.qr(rng.standard_normal((m, r)))[0]
    Q2 = np.linalg.qr(rng.standard_normal((n, r)))[0]
    return (Q1 * np.asarray(s, float)) @ Q2.T


def lapack_xi_rank(A, xi):
    """The rule of Eq. (1) on numpy's (LAPACK's) singular values."""
    s2 = np.linalg.svd(A, compute_uv=False) ** 2
    return int(np.searchsorted(np.cumsum(s2) >= xi * s2.sum(), True) + 1)


# Three 8 x 5 blocks with exact spectra; squared values and running sums:
#   [3,2,1,1,1]: 9 13 14 15 16    [5,1,1,1,1]: 25 26 27 28 29    [2,1,1,1,1]: 4 5 6 7 8
SPECTRA = [[3, 2, 1, 1, 1], [5, 1, 1, 1, 1], [2, 1, 1, 1, 1]]
# expected k_i with the cap k = 3, worked out by hand from the running sums
EXPECTED = {0.55: [1, 1, 2], 0.7: [2, 1, 3], 0.9: [3, 3, 3], 0.0: [3, 3, 3]}


def spectra_matrix(seed=5):
    rng = np.random.default_rng(seed)
    return np.vstack([prescribed(8, 5, s, rng) for s in SPECTRA])


def test_xi_rank_closed_form(orc):
    s = [3.0, 2.0, 1.0, 1.0, 1.0]                 # squares 9 4 1 1 1, total 16
    assert orc.xi_rank(s, 0.5) == 1               # 9 >= 8
    assert orc.xi_rank(s, 0.8125) == 2            # 13 >= 13 exactly: ">=" holds
    assert orc.xi_rank(s, 0.82) == 3
    assert orc.xi_rank(s, 0.99) == 5
    assert orc.xi_rank(s, 0.0) == 5 and orc.xi_rank(s, 1.0) == 5   # rule off
    assert orc.xi_rank([0.0, 0.0], 0.5) == 2


@pytest.mark.parametrize("xi", sorted(EXPECTED))
def test_store_ranks_on_prescribed_spectra(orc, xi):
    A = spectra_matrix()
    st = orc.store(A, 8, 3, xi=xi)
    assert list(st.k_i) == EXPECTED[xi]
    for i, ki in enumerate(st.k_i):
        assert np.allclose(st.S[i, :ki], SPECTRA[i][:ki], rtol=1e-12)
        assert np.all(st.S[i, ki:] == 0.0)
        assert np.all(st.U[i * 8:(i + 1) * 8, ki:] == 0.0) and np.all(st.V[i][:, ki:] == 0.0)


def test_store_ranks_match_lapack(orc):
    ser = synth.sinusoid_mixture(3_000, 12, sources=5, seed=41, noise="iid", noise_sigma=0.3)
    A, b, k = ser.A, 250, 12
    for xi in (0.6, 0.9, 0.98, 0.999):
        st = orc.store(A, b, k, xi=xi)
        for i in range(st.nb):
            blk = A[i * b:(i + 1) * b]
            assert st.k_i[i] == min(k, lapack_xi_rank(blk, xi)), (xi, i)


def test_partial_svd_rank_matches_lapack(orc):
    rng = np.random.default_rng(9)
    A = prescribed(40, 6, [9.0, 4.0, 2.0, 1.5, 1.0, 0.5], rng)
    base = orc.store(A, 40, 6)                  # exact: k = c = rank
    for xi in (0.7, 0.9, 0.97):
        st = orc.store_from_arrays(base.t, base.c, base.b, base.k, base.U, base.S, base.V,
                                   base.k_i, xi=xi)
        for r0, r1 in [(0, 17), (5, 40), (11, 29)]:
            Up, sp, Vp, rank = orc.partial_svd(st, 0, r0, r1)
            want = lapack_xi_rank(A[r0:r1], xi)
            assert rank == want, (xi, r0, r1)
            ref = np.linalg.svd(A[r0:r1], compute_uv=False)
            assert np.allclose(sp[:rank], ref[:rank], rtol=1e-11)
            assert np.all(sp[rank:] == 0.0) and np.all(Up[:, rank:] == 0.0)
            assert np.all(Vp[:, rank:] == 0.0)


def test_query_rank_on_exact_low_rank_blocks(orc):
    """Blocks of rank 2 with equal singular values keep both for 1/2 < xi < 1, so
    a range of whole blocks stitches exactly; its xi rank is that of the
    direct SVD of the range."""
    rng = np.random.default_rng(13)
    A = np.vstack([prescribed(10, 6, [s, s], rng) for s in (3.0, 1.0, 2.0, 0.5)])
    for xi in (0.6, 0.8, 0.95, 0.995):
        st = orc.store(A, 10, 6, xi=xi)
        assert list(st.k_i) == [2, 2, 2, 2]
        for ts, te in [(0, 40), (10, 30), (20, 40)]:
            U, s, V, ko = orc.query(st, ts, te, 6)
            assert ko == lapack_xi_rank(A[ts:te], xi), (xi, ts, te)
            ref = np.linalg.svd(A[ts:te], compute_uv=False)
            assert np.allclose(s[:ko], ref[:ko], rtol=1e-11)
            assert np.all(s[ko:] == 0.0) and np.all(U[:, ko:] == 0.0)


def test_xi_off_reproduces_fixed_rank(orc):
    ser = synth.sinusoid_mixture(2_000, 10, sources=4, seed=3, noise="iid", noise_sigma=0.1)
    ref = orc.store(ser.A, 300, 6)
    for xi in (0.0, 1.0):
        st = orc.store(ser.A, 300, 6, xi=xi)
        for a, b in ((st.U, ref.U), (st.S, ref.S), (st.V, ref.V), (st.k_i, ref.k_i)):
            np.testing.assert_array_equal(a, b)
        q = orc.query(st, 123, 1_777, 6)
        r = orc.query(ref, 123, 1_777, 6)
        for a, b in zip(q[:3], r[:3]):
            np.testing.assert_array_equal(a, b)


def test_ranks_grow_with_xi(orc):
    ser = synth.sinusoid_mixture(2_400, 16, sources=6, seed=8, noise="ar1", noise_sigma=0.05)
    prev = None
    for xi in (0.3, 0.6, 0.8, 0.9, 0.95, 0.99, 0.999):
        st = orc.store(ser.A, 400, 16, xi=xi)
        ks = np.array([orc.query(st, 37, 2_301, 16)[3]] + list(st.k_i))
        if prev is not None:
            assert np.all(ks >= prev)
        prev = ks


# ------------------------------------------------ planted mistakes are caught
MUTANTS = {
    "strict_inequality": ("if (run >= xi * total) return j + 1;",
                          "if (run > xi * total) return j + 1;"),
    "sigma_not_squared": ("run += s[j] * s[j];", "run += s[j] * (s[j] > 0.0 ? 1.0 : 0.0);"),
    "store_total_of_top_k": ("const int64_t kx = zo_xi_rank(sb, r, xi);",
                             "const int64_t kx = zo_xi_rank(sb, k < r ? k : r, xi);"),
    "partial_ignores_xi": ("const int64_t kx = zo_xi_rank(sp, rp, xi);", "const int64_t kx = rp;"),
    "query_ignores_xi": ("const int64_t kx = zo_xi_rank(sr, r, xi);", "const int64_t kx = r;"),
}

PIN_SCRIPT = textwrap.dedent(r'''
    import sys
    sys.path.insert(0, {root!r})
    import oracle
    from tests import test_oracle_xi as T

    class Orc:
        def __getattr__(self, n):
            f = getattr(oracle, n)
            if n in ("xi_rank", "store", "partial_svd", "query"):
                return lambda *a, **kw: f(*a, lib=LIB, **kw)
            return f
    LIB = oracle.load({lib!r})
    orc = Orc()
    try:
        T.test_xi_rank_closed_form(orc)
        for xi in sorted(T.EXPECTED):
            T.test_store_ranks_on_prescribed_spectra(orc, xi)
        T.test_partial_svd_rank_matches_lapack(orc)
        T.test_query_rank_on_exact_low_rank_blocks(orc)
    except Exception as e:
        print("PIN FAILED:", type(e).__name__, e)
        sys.exit(3)
    print("ALL PINS PASSED")
''')


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_xi_mistake_is_caught(orc, tmp_path, name):
    old, new = MUTANTS[name]
    src = open(os.path.join(ROOT, "oracle", "zoom_oracle.c")).read()
    assert src.count(old) == 1, "mutation anchor missing: " + name
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new))
    lib = str(tmp_path / "libmutant.so")
    orc.build(force=True, src=str(mut), out=lib)
    script = tmp_path / "pins.py"
    script.write_text(PIN_SCRIPT.format(root=ROOT, lib=lib))
    r = subprocess.run([sys.executable, str(script)], capture_output=True, text=True, timeout=120,
                       env=dict(os.environ, OMP_NUM_THREADS="2"), cwd=ROOT)
    assert "ALL PINS PASSED" not in r.stdout, "planted mistake %s went unnoticed" % name


def test_unmutated_oracle_passes_xi_pin_script(orc, tmp_path):
    script = tmp_path / "pins.py"
    script.write_text(PIN_SCRIPT.format(root=ROOT, lib=os.path.join(ROOT, "oracle", "liboracle.so")))
    r = subprocess.run([sys.executable, str(script)], capture_output=True, text=True, timeout=120,
                       cwd=ROOT)
    assert "ALL PINS PASSED" in r.stdout, r.stdout + r.stderr
