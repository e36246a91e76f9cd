"""CPU FP64 oracle for Zoom-SVD (arXiv 1805.00754).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that the
GPU library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code
with the HIP library and imports nothing from the product package.

The arithmetic lives in ``zoom_oracle.c`` (plain C, double precision, no
vendor BLAS); this module compiles it with gcc and exposes it through ctypes
with numpy arrays.  Conventions: row-major arrays, 0-based half-open time
ranges ``[t_s, t_e)``, block ``i`` = rows ``[i*b, min((i+1)*b, t))``.

Parity pins for every function here live in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "zoom_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

# Numerical-rank threshold, relative to sigma_1 of the matrix being
# decomposed.  The paper does not fix one; singular values below this
# fraction of sigma_1 are taken as numerically zero.
RANK_TOL = 1e-11

CFLAGS = ["-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared"]


def build(force: bool = True, src: str = _SRC, out: str = _LIB) -> str:
    """Compile the oracle with gcc.  Returns the path of the shared object."""
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dbl = ctypes.c_double
_pd = ctypes.POINTER(ctypes.c_double)
_pi64 = ctypes.POINTER(ctypes.c_int64)
_pi32 = ctypes.POINTER(ctypes.c_int32)


def load(path: str | None = None):
    """Load (building first if needed) the oracle library."""
    global _lib
    with _lock:
        if path is not None:
            return _bind(ctypes.CDLL(path))
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            _lib = _bind(ctypes.CDLL(_LIB))
        return _lib


def _bind(lib):
    lib.zo_svd.argtypes = [_i64, _i64, _pd, _i64, _dbl, _i64, _pd, _i64, _pd, _pd, _i64, _pi32]
    lib.zo_svd.restype = ctypes.c_int
    lib.zo_store.argtypes = [_pd, _i64, _i64, _i64, _i64, _i32, _dbl, _dbl, _pd, _pd, _pd, _pi32]
    lib.zo_store.restype = ctypes.c_int
    lib.zo_partial_svd.argtypes = [_pd, _pd, _pd, _i64, _i64, _i32, _i64, _i64, _i64, _dbl,
                                   _dbl, _pd, _pd, _pd, _pi32]
    lib.zo_partial_svd.restype = ctypes.c_int
    lib.zo_query.argtypes = [_pd, _pd, _pd, _i64, _i64, _i64, _i32, _i64, _i64, _i32, _dbl,
                             _dbl, _pd, _pd, _pd, _pi32]
    lib.zo_query.restype = ctypes.c_int
    lib.zo_query_batch.argtypes = [_pd, _pd, _pd, _i64, _i64, _i64, _i32, _i32, _pi64, _pi64,
                                   _pi32, _dbl, _dbl, _pd, _pi64, _pd, _pi64, _pd, _pi64, _pi32]
    lib.zo_query_batch.restype = ctypes.c_int
    lib.zo_direct.argtypes = [_pd, _i64, _i64, _i64, _i64, _i32, _dbl, _pd, _pd, _pd, _pi32]
    lib.zo_direct.restype = ctypes.c_int
    lib.zo_query_blocks.argtypes = [_i64, _i64, _i64, _pi64, _pi64, _pi64, _pi64]
    lib.zo_query_blocks.restype = None
    lib.zo_num_blocks.argtypes = [_i64, _i64]
    lib.zo_num_blocks.restype = _i64
    lib.zo_block_rows.argtypes = [_i64, _i64, _i64]
    lib.zo_block_rows.restype = _i64
    lib.zo_xi_rank.argtypes = [_pd, _i64, _dbl]
    lib.zo_xi_rank.restype = _i64
    lib.zo_direct_batch.argtypes = [_pd, _i64, _i64, _i32, _pi64, _pi64, _pi32, _dbl, _pd, _pi64,
                                    _pd, _pi64, _pd, _pi64, _pi32]
    lib.zo_direct_batch.restype = ctypes.c_int
    lib.zo_set_threads.argtypes = [ctypes.c_int]
    lib.zo_set_threads.restype = None
    lib.zo_max_threads.argtypes = []
    lib.zo_max_threads.restype = ctypes.c_int
    return lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    if a.dtype == np.float64:
        return a.ctypes.data_as(_pd)
    if a.dtype == np.int64:
        return a.ctypes.data_as(_pi64)
    if a.dtype == np.int32:
        return a.ctypes.data_as(_pi32)
    raise TypeError(a.dtype)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    pass


def svd(A, rank_tol: float = RANK_TOL, nvec: int | None = None, lib=None):
    """Thin SVD (Sec. 2.1).  Returns (U m x r, s r, V n x r, rank, sweeps)."""
    lib = lib or load()
    A = _f64(np.atleast_2d(A))
    m, n = A.shape
    r = min(m, n)
    nvec = r if nvec is None else min(nvec, r)
    U = np.zeros((m, r))
    s = np.zeros(r)
    V = np.zeros((n, r))
    rank = np.zeros(1, np.int32)
    sweeps = lib.zo_svd(m, n, _p(A), n, rank_tol, nvec, _p(U), r, _p(s), _p(V), r, _p(rank))
    return U, s, V, int(rank[0]), int(sweeps)


class Store:
    """Blocks compressed by the oracle's storage phase (Def. 2 sets U, S, V).

    U: t x k (rows of block i hold U_(i)), S: nb x k, V: nb x c x k, k_i: nb.
    xi: the energy threshold of Eq. (1) (0: none), also applied by the query
    phase to the Partial-SVD and to the stacked SVD.
    """

    def __init__(self, t, c, b, k, U, S, V, k_i, rank_tol, xi=0.0):
        self.t, self.c, self.b, self.k = int(t), int(c), int(b), int(k)
        self.U, self.S, self.V, self.k_i = U, S, V, k_i
        self.rank_tol = rank_tol
        self.xi = float(xi)

    @property
    def nb(self) -> int:
        return int(self.S.shape[0])

    def block_rows(self, i: int) -> int:
        return min(self.b, self.t - i * self.b)

    def stored_elements(self) -> int:
        """Elements a store of exactly the kept triplets needs: sum k_i (b_i + 1 + c)."""
        return int(sum(int(self.k_i[i]) * (self.block_rows(i) + 1 + self.c) for i in range(self.nb)))


def store(A, b: int, k: int, rank_tol: float = RANK_TOL, lib=None, xi: float = 0.0) -> Store:
    """Storage phase, batch form (Alg. 1 / Def. 1 / Def. 2); with 0 < xi < 1
    block i keeps k_i = min(k, numerical rank, xi rank of Eq. (1))."""
    lib = lib or load()
    A = _f64(A)
    t, c = A.shape
    nb = (t + b - 1) // b
    U = np.zeros((t, k))
    S = np.zeros((nb, k))
    V = np.zeros((nb, c, k))
    k_i = np.zeros(nb, np.int32)
    bad = lib.zo_store(_p(A), t, c, c, b, k, rank_tol, xi, _p(U), _p(S), _p(V), _p(k_i))
    if bad:
        raise OracleError("Jacobi did not converge on %d blocks" % bad)
    return Store(t, c, b, k, U, S, V, k_i, rank_tol, xi)


def append(st: Store, R, lib=None) -> Store:
    """Streaming ingest (Alg. 1's incremental update, Eqs. (2)-(3), for the
    appended rows at once): the rows first fill the last block,
        [U S V^T; R1] = diag(U, I) [S V^T; R1],  [S V^T; R1] = U' S' V'^T,
    the last block becoming diag(U, I) U', S', V' (truncated as any block);
    the remaining rows form new blocks as in the storage phase.  Returns a new
    Store of t + m rows."""
    lib = lib or load()
    R = _f64(R)
    m = R.shape[0]
    t0, b, k, c = st.t, st.b, st.k, st.c
    nb0 = st.nb
    r_tail = t0 - (nb0 - 1) * b
    m1 = min(m, b - r_tail) if r_tail < b else 0
    U = [st.U]
    S, V, k_i = st.S.copy(), st.V.copy(), st.k_i.copy()
    if m1:
        i = nb0 - 1
        P = np.vstack([st.S[i][:, None] * st.V[i].T, R[:m1]])       # (k + m1) x c
        tp = store(P, k + m1, k, rank_tol=st.rank_tol, lib=lib, xi=st.xi)
        Ut = np.vstack([st.U[i * b:i * b + r_tail] @ tp.U[:k], tp.U[k:]])
        U = [st.U[:i * b], Ut]
        S[i], V[i], k_i[i] = tp.S[0], tp.V[0], tp.k_i[0]
    if m > m1:
        nst = store(R[m1:], b, k, rank_tol=st.rank_tol, lib=lib, xi=st.xi)
        U.append(nst.U)
        S = np.concatenate([S, nst.S])
        V = np.concatenate([V, nst.V])
        k_i = np.concatenate([k_i, nst.k_i])
    return Store(t0 + m, c, b, k, np.ascontiguousarray(np.vstack(U)), np.ascontiguousarray(S),
                 np.ascontiguousarray(V), np.ascontiguousarray(k_i, np.int32), st.rank_tol, st.xi)


def store_from_arrays(t, c, b, k, U, S, V, k_i=None, rank_tol: float = RANK_TOL,
                      xi: float = 0.0) -> Store:
    """Wrap block factors produced elsewhere (e.g. downloaded from the GPU)
    so that the oracle's query phase can run on them."""
    U = _f64(U).reshape(t, k)
    S = _f64(S).reshape(-1, k)
    V = _f64(V).reshape(-1, c, k)
    if k_i is None:
        k_i = (S > 0).sum(axis=1).astype(np.int32)
    return Store(t, c, b, k, U, S, V, np.ascontiguousarray(k_i, np.int32), rank_tol, xi)


def partial_svd(st: Store, i: int, r0: int, r1: int, lib=None):
    """Partial-SVD of block i restricted to rows [r0, r1) (Alg. 3).
    Returns (U' m x rp, Sigma' rp, V' c x rp, rank)."""
    lib = lib or load()
    m = r1 - r0
    rp = min(m, st.k)
    Up = np.zeros((m, rp))
    sp = np.zeros(rp)
    Vp = np.zeros((st.c, rp))
    rank = np.zeros(1, np.int32)
    sw = lib.zo_partial_svd(_p(st.U), _p(st.S), _p(st.V), st.c, st.b, st.k, i, r0, r1,
                            st.rank_tol, st.xi, _p(Up), _p(sp), _p(Vp), _p(rank))
    if sw < 0:
        raise OracleError("Jacobi did not converge")
    return Up, sp, Vp, int(rank[0])


def xi_rank(s, xi: float, lib=None) -> int:
    """Eq. (1): the smallest k with sum_{j<k} s_j^2 >= xi sum_j s_j^2 over all
    the singular values s (descending); len(s) when 0 < xi < 1 does not hold."""
    lib = lib or load()
    s = _f64(np.asarray(s, np.float64).ravel())
    return int(lib.zo_xi_rank(_p(s), len(s), float(xi)))


def query_blocks(t_s: int, t_e: int, b: int, lib=None):
    """Alg. 3 index math for [t_s, t_e): returns (S, E, lo, hi)."""
    lib = lib or load()
    out = [np.zeros(1, np.int64) for _ in range(4)]
    lib.zo_query_blocks(t_s, t_e, b, *[_p(o) for o in out])
    return tuple(int(o[0]) for o in out)


def query(st: Store, t_s: int, t_e: int, kq: int, lib=None):
    """Query phase (Alg. 2).  Returns (U n x kq, s kq, V c x kq, k_out)."""
    lib = lib or load()
    if not (0 <= t_s < t_e <= st.t) or not (1 <= kq <= st.k):
        raise ValueError("bad query")
    n = t_e - t_s
    U = np.zeros((n, kq))
    s = np.zeros(kq)
    V = np.zeros((st.c, kq))
    kout = np.zeros(1, np.int32)
    bad = lib.zo_query(_p(st.U), _p(st.S), _p(st.V), st.t, st.c, st.b, st.k, t_s, t_e, kq,
                       st.rank_tol, st.xi, _p(U), _p(s), _p(V), _p(kout))
    if bad:
        raise OracleError("Jacobi did not converge")
    return U, s, V, int(kout[0])


def query_batch(st: Store, ts, te, kq, lib=None, with_u: bool = True):
    """Many queries, parallel over queries (OpenMP).  Returns a list of
    (U, s, V, k_out) tuples, one per query.  with_u=False skips the
    block-diagonal product of Eq. (9) (U is then None): Sigma and V of very
    tall ranges without their n x k_q left factors."""
    lib = lib or load()
    ts = np.ascontiguousarray(ts, np.int64)
    te = np.ascontiguousarray(te, np.int64)
    kq = np.ascontiguousarray(np.broadcast_to(kq, ts.shape), np.int32)
    nq = len(ts)
    n = te - ts
    uoff = np.zeros(nq, np.int64)
    voff = np.zeros(nq, np.int64)
    soff = np.zeros(nq, np.int64)
    if nq:
        uoff[1:] = np.cumsum(n * kq)[:-1]
        voff[1:] = np.cumsum(np.full(nq, st.c) * kq)[:-1]
        soff[1:] = np.cumsum(kq)[:-1]
    U = np.zeros(int((n * kq).sum()) if with_u else 1)
    V = np.zeros(int(st.c * kq.sum()))
    s = np.zeros(int(kq.sum()))
    kout = np.zeros(nq, np.int32)
    bad = lib.zo_query_batch(_p(st.U), _p(st.S), _p(st.V), st.t, st.c, st.b, st.k, nq, _p(ts),
                             _p(te), _p(kq), st.rank_tol, st.xi, _p(U) if with_u else None,
                             _p(uoff), _p(s), _p(soff), _p(V), _p(voff), _p(kout))
    if bad:
        raise OracleError("Jacobi did not converge in %d queries" % bad)
    res = []
    for q in range(nq):
        res.append((U[uoff[q]:uoff[q] + n[q] * kq[q]].reshape(n[q], kq[q]) if with_u else None,
                    s[soff[q]:soff[q] + kq[q]],
                    V[voff[q]:voff[q] + st.c * kq[q]].reshape(st.c, kq[q]),
                    int(kout[q])))
    return res


def window_similarity(st: Store, t_s: int, t_e: int, stride: int, n_windows: int, lib=None):
    """The case study of Sec. 5 (finding similar time ranges): u_1 of the base
    range [t_s, t_e) and of every earlier window [t_s - w stride, t_e - w
    stride), w = 1..n_windows, each from the query phase at rank 1; returns
    the cosines <u_base, u_w> / (|u_base| |u_w|) (0 for a zero vector)."""
    u0 = query(st, t_s, t_e, 1, lib=lib)[0][:, 0]
    out = np.zeros(n_windows)
    for w in range(1, n_windows + 1):
        uw = query(st, t_s - w * stride, t_e - w * stride, 1, lib=lib)[0][:, 0]
        den = np.linalg.norm(u0) * np.linalg.norm(uw)
        out[w - 1] = float(u0 @ uw) / den if den > 0 else 0.0
    return out


def direct(A, t_s: int, t_e: int, kq: int, rank_tol: float = RANK_TOL, lib=None):
    """SVD of the raw rows A[t_s:t_e) truncated to kq (Problem 1)."""
    lib = lib or load()
    A = _f64(A)
    c = A.shape[1]
    n = t_e - t_s
    U = np.zeros((n, kq))
    s = np.zeros(kq)
    V = np.zeros((c, kq))
    kout = np.zeros(1, np.int32)
    bad = lib.zo_direct(_p(A), c, c, t_s, t_e, kq, rank_tol, _p(U), _p(s), _p(V), _p(kout))
    if bad:
        raise OracleError("Jacobi did not converge")
    return U, s, V, int(kout[0])


def direct_batch(A, ts, te, kq, rank_tol: float = RANK_TOL, lib=None):
    """direct() for many ranges of one matrix, parallel over ranges (OpenMP).
    Returns a list of (U, s, V, k_out) tuples, one per range."""
    lib = lib or load()
    A = _f64(A)
    c = A.shape[1]
    ts = np.ascontiguousarray(ts, np.int64)
    te = np.ascontiguousarray(te, np.int64)
    kq = np.ascontiguousarray(np.broadcast_to(kq, ts.shape), np.int32)
    nq = len(ts)
    n = te - ts
    uoff = np.zeros(nq, np.int64)
    voff = np.zeros(nq, np.int64)
    soff = np.zeros(nq, np.int64)
    if nq:
        uoff[1:] = np.cumsum(n * kq)[:-1]
        voff[1:] = np.cumsum(np.full(nq, c) * kq)[:-1]
        soff[1:] = np.cumsum(kq)[:-1]
    U = np.zeros(int((n * kq).sum()))
    V = np.zeros(int(c * kq.sum()))
    s = np.zeros(int(kq.sum()))
    kout = np.zeros(nq, np.int32)
    bad = lib.zo_direct_batch(_p(A), c, c, nq, _p(ts), _p(te), _p(kq), rank_tol, _p(U), _p(uoff),
                              _p(s), _p(soff), _p(V), _p(voff), _p(kout))
    if bad:
        raise OracleError("Jacobi did not converge in %d ranges" % bad)
    return [(U[uoff[q]:uoff[q] + n[q] * kq[q]].reshape(n[q], kq[q]), s[soff[q]:soff[q] + kq[q]],
             V[voff[q]:voff[q] + c * kq[q]].reshape(c, kq[q]), int(kout[q])) for q in range(nq)]


def set_threads(n: int, lib=None) -> None:
    """Number of OpenMP threads of the oracle's parallel loops."""
    (lib or load()).zo_set_threads(int(n))


def max_threads(lib=None) -> int:
    lib = lib or load()
    return int(lib.zo_max_threads())
