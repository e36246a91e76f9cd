"""Python binding of the Zoom-SVD C ABI (include/zoomsvd.h).

Argument marshalling only: every step of the method runs in the HIP library
``libzoomsvd.so`` built from ``csrc/``.  PyTorch supplies device memory and
streams.  If the library is missing this module raises on first use; there is
no fallback path.

Names follow the C ABI: ``zs_store_blocks``, ``zs_query``, ``zs_query_batch``,
``zs_query_batch_graph``, ``zs_store_get_block``, ``zs_store_bytes``,
``zs_sync_status``, ...
Time ranges are 0-based half-open ``[t_s, t_e)``.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np
import torch  # loads the HIP runtime the library binds to

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libzoomsvd.so")

ZS_OK, ZS_EINVAL, ZS_ERANGE, ZS_ENOMEM, ZS_ENOCONV, ZS_EDEVICE, ZS_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
ZS_F64, ZS_F32, ZS_BF16 = 0, 1, 2
ZS_MODE_FP64, ZS_MODE_FP32, ZS_MODE_BF16 = 0, 1, 2
STATUS_NAMES = {0: "ZS_OK", -1: "ZS_EINVAL", -2: "ZS_ERANGE", -3: "ZS_ENOMEM", -4: "ZS_ENOCONV",
                -5: "ZS_EDEVICE", -6: "ZS_EUNSUPPORTED"}

# Symbols the header declares (the CPU test checks the library exports all).
EXPORTED = ["zs_store_blocks", "zs_store_blocks_xi", "zs_store_append", "zs_window_similarity",
            "zs_query", "zs_query_noalloc", "zs_query_scratch_bytes", "zs_query_batch",
            "zs_query_batch_graph",
            "zs_batch_graph_launch", "zs_batch_graph_free", "zs_store_graph_create",
            "zs_store_graph_launch", "zs_store_graph_free", "zs_store_free", "zs_release_workspaces",
            "zs_store_bytes",
            "zs_store_info", "zs_store_get_block", "zs_sync_status", "zs_last_error", "zs_version",
            "zs_timing_enable", "zs_timing_reset", "zs_timing_get", "zs_set_sweep_cap", "zs_autotune",
            "zs_autotune_force", "zs_autotune_table"]


class ZSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


_lock = threading.Lock()
_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32


def load(path: str | None = None):
    """Load libzoomsvd.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is not None and path is None:
            return _lib
        p = path or LIB_PATH
        if not os.path.exists(p):
            raise RuntimeError("libzoomsvd.so not built: run `python -m paper_1805_00754_amd.build` "
                               "(expected at %s)" % p)
        lib = ctypes.CDLL(p)
        lib.zs_store_blocks.argtypes = [_vp, _i64, _i64, _i64, ctypes.c_int, _i64, _i32,
                                        ctypes.c_int, _vp, ctypes.POINTER(_vp)]
        lib.zs_store_blocks_xi.argtypes = [_vp, _i64, _i64, _i64, ctypes.c_int, _i64, _i32,
                                           ctypes.c_int, ctypes.c_double, _vp, ctypes.POINTER(_vp)]
        lib.zs_query.argtypes = [_vp, _i64, _i64, _i32, _vp, _i64, _vp, _vp, _i64, _vp, _vp]
        lib.zs_query_noalloc.argtypes = lib.zs_query.argtypes
        lib.zs_query_scratch_bytes.argtypes = [_vp, _i64, _i64, _i32]
        lib.zs_query_scratch_bytes.restype = _i64
        lib.zs_window_similarity.argtypes = [_vp, _i64, _i64, _i64, _i32, _vp, _vp]
        lib.zs_store_append.argtypes = [_vp, _vp, _i64, _i64, ctypes.c_int, _vp]
        lib.zs_query_batch.argtypes = [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                       _vp, _vp]
        lib.zs_query_batch_graph.argtypes = [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                             _vp, _vp, _vp, ctypes.POINTER(_vp)]
        lib.zs_batch_graph_launch.argtypes = [_vp, _vp]
        lib.zs_store_graph_create.argtypes = [_vp, _i64, _i64, _i64, ctypes.c_int, _i64, _i32,
                                              ctypes.c_int, _vp, ctypes.POINTER(_vp),
                                              ctypes.POINTER(_vp)]
        lib.zs_store_graph_launch.argtypes = [_vp, _vp]
        lib.zs_store_graph_free.argtypes = [_vp]
        lib.zs_store_graph_free.restype = None
        lib.zs_batch_graph_free.argtypes = [_vp]
        lib.zs_batch_graph_free.restype = None
        lib.zs_store_free.argtypes = [_vp]
        lib.zs_store_free.restype = None
        lib.zs_store_bytes.argtypes = [_vp]
        lib.zs_store_bytes.restype = _i64
        lib.zs_store_info.argtypes = [_vp] + [_vp] * 6
        lib.zs_store_get_block.argtypes = [_vp, _i64, _vp, _vp, _vp, _vp, _vp]
        lib.zs_sync_status.argtypes = [_vp, _vp]
        lib.zs_release_workspaces.argtypes = [_vp]
        lib.zs_last_error.restype = ctypes.c_char_p
        lib.zs_version.restype = ctypes.c_char_p
        lib.zs_timing_enable.argtypes = [ctypes.c_int]
        lib.zs_timing_enable.restype = None
        lib.zs_timing_reset.restype = None
        lib.zs_timing_get.argtypes = [ctypes.c_char_p, _vp, _vp]
        lib.zs_set_sweep_cap.argtypes = [ctypes.c_int]
        lib.zs_set_sweep_cap.restype = ctypes.c_int
        lib.zs_autotune.argtypes = [ctypes.c_int]
        lib.zs_autotune.restype = None
        lib.zs_autotune_force.argtypes = [ctypes.c_char_p, ctypes.c_int]
        lib.zs_autotune_force.restype = ctypes.c_int
        lib.zs_autotune_table.restype = ctypes.c_char_p
        for name in ("zs_store_blocks", "zs_store_blocks_xi", "zs_store_append",
                     "zs_window_similarity", "zs_query", "zs_query_noalloc", "zs_query_batch",
                     "zs_store_info",
                     "zs_store_get_block", "zs_sync_status", "zs_timing_get",
                     "zs_query_batch_graph", "zs_batch_graph_launch", "zs_store_graph_create",
                     "zs_store_graph_launch", "zs_release_workspaces"):
            getattr(lib, name).restype = ctypes.c_int
        if path is None:
            _lib = lib
        return lib


def zs_last_error() -> str:
    return load().zs_last_error().decode()


def zs_version() -> str:
    return load().zs_version().decode()


def _check(status: int):
    if status != ZS_OK:
        raise ZSError(status, zs_last_error())


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def _ptr(t: torch.Tensor) -> int:
    return int(t.data_ptr())


class Store:
    """A device-resident store (Def. 2 sets U, S, V) owned by the library."""

    def __init__(self, handle: int, t: int, c: int, b: int, k: int, mode: int, xi: float = 0.0):
        self.handle = handle
        self.t, self.c, self.b, self.k, self.mode = t, c, b, k, mode
        self.xi = xi
        self.nb = (t + b - 1) // b

    def block_rows(self, i: int) -> int:
        return min(self.b, self.t - i * self.b)

    def free(self):
        if self.handle:
            load().zs_store_free(_vp(self.handle))
            self.handle = 0

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    @property
    def out_dtype(self):
        return torch.float64 if self.mode == ZS_MODE_FP64 else torch.float32


def zs_store_blocks(A: torch.Tensor, b: int, k: int, mode: int = ZS_MODE_FP64, stream=None,
                    xi: float = 0.0) -> Store:
    """Storage phase: compress every b-row block of A (t x c, on the GPU) to
    its rank-k SVD (zs_store_blocks), or with 0 < xi < 1 to the rank of the
    energy threshold of Eq. (1) capped at k (zs_store_blocks_xi; queries on the
    store then apply the same rule).  Raises ZSError on failure (ZS_ENOCONV
    still leaves the error raised; the store is freed)."""
    if A.dim() != 2 or A.stride(1) != 1 or not A.is_cuda:
        raise ValueError("A must be a 2-D CUDA/HIP tensor with unit column stride")
    a_type = {torch.float64: ZS_F64, torch.float32: ZS_F32, torch.bfloat16: ZS_BF16}[A.dtype]
    t, c = A.shape
    h = _vp()
    if xi:
        st = load().zs_store_blocks_xi(_vp(_ptr(A)), t, c, A.stride(0), a_type, b, k, mode,
                                       float(xi), _vp(_stream(stream)), ctypes.byref(h))
    else:
        st = load().zs_store_blocks(_vp(_ptr(A)), t, c, A.stride(0), a_type, b, k, mode,
                                    _vp(_stream(stream)), ctypes.byref(h))
    if st == ZS_ENOCONV and h.value:
        load().zs_store_free(h)
    _check(st)
    return Store(h.value, t, c, b, k, mode, float(xi))


class StoreGraph:
    """The storage phase of a fixed input captured into a HIP graph
    (zs_store_graph_create): launch() recompresses the input's current
    contents into the same store.  Keeps the input tensor alive."""

    def __init__(self, st: Store, A: torch.Tensor, handle):
        self.st = st
        self.A = A
        self.handle = handle

    def launch(self, stream=None):
        _check(load().zs_store_graph_launch(_vp(self.handle), _vp(_stream(stream))))

    def free(self):
        if self.handle:
            load().zs_store_graph_free(_vp(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def zs_store_graph_create(A: torch.Tensor, b: int, k: int, mode: int = ZS_MODE_FP64,
                          stream=None) -> StoreGraph:
    """Builds the store of A (t x c, on the GPU) and captures its storage phase
    into a graph; returns the StoreGraph (its .st is the store).  Free the
    graph before the store."""
    if A.dim() != 2 or A.stride(1) != 1 or not A.is_cuda:
        raise ValueError("A must be a 2-D CUDA/HIP tensor with unit column stride")
    a_type = {torch.float64: ZS_F64, torch.float32: ZS_F32, torch.bfloat16: ZS_BF16}[A.dtype]
    t, c = A.shape
    hs, hg = _vp(), _vp()
    s = load().zs_store_graph_create(_vp(_ptr(A)), t, c, A.stride(0), a_type, b, k, mode,
                                     _vp(_stream(stream)), ctypes.byref(hs), ctypes.byref(hg))
    if s == ZS_ENOCONV and hg.value:
        load().zs_store_graph_free(hg)
        load().zs_store_free(hs)
    _check(s)
    return StoreGraph(Store(hs.value, t, c, b, k, mode), A, hg.value)


def zs_store_append(st: Store, R: torch.Tensor, stream=None) -> Store:
    """Streaming ingest: append the rows of R (m x c, on the GPU) to the store
    (its last block by the incremental update, then new blocks).  Updates
    st.t and st.nb; returns st."""
    if R.dim() != 2 or R.stride(1) != 1 or not R.is_cuda or R.shape[1] != st.c:
        raise ValueError("R must be a 2-D CUDA/HIP tensor of c columns with unit column stride")
    r_type = {torch.float64: ZS_F64, torch.float32: ZS_F32, torch.bfloat16: ZS_BF16}[R.dtype]
    s = load().zs_store_append(_vp(st.handle), _vp(_ptr(R)), R.shape[0], R.stride(0), r_type,
                               _vp(_stream(stream)))
    if s in (ZS_OK, ZS_ENOCONV):
        st.t += R.shape[0]
        st.nb = (st.t + st.b - 1) // st.b
    _check(s)
    return st


def zs_query(st: Store, t_s: int, t_e: int, k_q: int, U=None, S=None, V=None, k_out=None,
             stream=None, noalloc: bool = False):
    """Query phase for [t_s, t_e).  Returns (U n x k_q, S k_q, V c x k_q,
    k_out) as device tensors (allocated when not given).  With noalloc the
    call goes to zs_query_noalloc (the library allocates nothing; its fixed
    scratch is shared by every such call on the device)."""
    dev = torch.device("cuda", torch.cuda.current_device())
    n = t_e - t_s
    if U is None:
        U = torch.empty((max(n, 0), k_q), dtype=st.out_dtype, device=dev)
    if S is None:
        S = torch.empty(k_q, dtype=torch.float64, device=dev)
    if V is None:
        V = torch.empty((st.c, k_q), dtype=st.out_dtype, device=dev)
    if k_out is None:
        k_out = torch.empty(1, dtype=torch.int32, device=dev)
    fn = load().zs_query_noalloc if noalloc else load().zs_query
    _check(fn(_vp(st.handle), t_s, t_e, k_q, _vp(_ptr(U)), U.stride(0), _vp(_ptr(S)), _vp(_ptr(V)),
              V.stride(0), _vp(_ptr(k_out)), _vp(_stream(stream))))
    return U, S, V, k_out


class Batch:
    """Output buffers of zs_query_batch with per-query views."""

    def __init__(self, st: Store, t_s, t_e, k_q, dev):
        self.t_s = np.ascontiguousarray(t_s, np.int64)
        self.t_e = np.ascontiguousarray(t_e, np.int64)
        self.k_q = np.ascontiguousarray(np.broadcast_to(k_q, self.t_s.shape), np.int32)
        nq = len(self.t_s)
        n = self.t_e - self.t_s
        self.u_off = np.zeros(nq, np.int64)
        self.s_off = np.zeros(nq, np.int64)
        self.v_off = np.zeros(nq, np.int64)
        if nq > 1:
            self.u_off[1:] = np.cumsum(n * self.k_q)[:-1]
            self.s_off[1:] = np.cumsum(self.k_q)[:-1]
            self.v_off[1:] = np.cumsum(st.c * self.k_q.astype(np.int64))[:-1]
        self.U = torch.empty(int((n * self.k_q).sum()), dtype=st.out_dtype, device=dev)
        self.S = torch.empty(int(self.k_q.sum()), dtype=torch.float64, device=dev)
        self.V = torch.empty(int(st.c * self.k_q.astype(np.int64).sum()), dtype=st.out_dtype,
                             device=dev)
        self.k_out = torch.empty(nq, dtype=torch.int32, device=dev)
        self.c = st.c

    def __len__(self):
        return len(self.t_s)

    def result(self, q: int):
        n = int(self.t_e[q] - self.t_s[q])
        kq = int(self.k_q[q])
        U = self.U[self.u_off[q]:self.u_off[q] + n * kq].view(n, kq)
        S = self.S[self.s_off[q]:self.s_off[q] + kq]
        V = self.V[self.v_off[q]:self.v_off[q] + self.c * kq].view(self.c, kq)
        return U, S, V, self.k_out[q:q + 1]


def zs_query_batch(st: Store, t_s, t_e, k_q, out: Batch | None = None, stream=None) -> Batch:
    """nq queries in one set of launches; returns a Batch of device buffers."""
    dev = torch.device("cuda", torch.cuda.current_device())
    if out is None:
        out = Batch(st, t_s, t_e, k_q, dev)
    nq = len(out)
    a = lambda x: _vp(x.ctypes.data)
    _check(load().zs_query_batch(_vp(st.handle), nq, a(out.t_s), a(out.t_e), a(out.k_q),
                                 _vp(_ptr(out.U)), a(out.u_off), _vp(_ptr(out.S)), a(out.s_off),
                                 _vp(_ptr(out.V)), a(out.v_off), _vp(_ptr(out.k_out)),
                                 _vp(_stream(stream))))
    return out


def zs_window_similarity(st: Store, t_s: int, t_e: int, stride: int, n_windows: int,
                         sim=None, stream=None) -> torch.Tensor:
    """Cosine of u_1 of each earlier window [t_s - w stride, t_e - w stride),
    w = 1..n_windows, with u_1 of the base range [t_s, t_e) (the case study of
    Sec. 5).  Returns a device tensor of n_windows doubles."""
    if sim is None:
        sim = torch.empty(n_windows, dtype=torch.float64,
                          device=torch.device("cuda", torch.cuda.current_device()))
    _check(load().zs_window_similarity(_vp(st.handle), t_s, t_e, stride, n_windows, _vp(_ptr(sim)),
                                       _vp(_stream(stream))))
    return sim


class BatchGraph:
    """A fixed batch captured into a HIP graph (zs_query_batch_graph).  Holds
    the store and the output Batch, which must outlive it."""

    def __init__(self, st: Store, out: Batch, handle):
        self.st = st
        self.out = out
        self.handle = handle

    def launch(self, stream=None):
        _check(load().zs_batch_graph_launch(_vp(self.handle), _vp(_stream(stream))))

    def free(self):
        if self.handle:
            load().zs_batch_graph_free(_vp(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def zs_query_batch_graph(st: Store, t_s, t_e, k_q, out: Batch | None = None,
                         stream=None) -> BatchGraph:
    """Plans the batch once, runs it eagerly (filling `out`) and captures its
    launches into a graph that replays them with BatchGraph.launch()."""
    dev = torch.device("cuda", torch.cuda.current_device())
    if out is None:
        out = Batch(st, t_s, t_e, k_q, dev)
    nq = len(out)
    a = lambda x: _vp(x.ctypes.data)
    h = _vp()
    _check(load().zs_query_batch_graph(_vp(st.handle), nq, a(out.t_s), a(out.t_e), a(out.k_q),
                                       _vp(_ptr(out.U)), a(out.u_off), _vp(_ptr(out.S)),
                                       a(out.s_off), _vp(_ptr(out.V)), a(out.v_off),
                                       _vp(_ptr(out.k_out)), _vp(_stream(stream)),
                                       ctypes.byref(h)))
    return BatchGraph(st, out, h.value)


def zs_query_batch_into(st: Store, t_s, t_e, k_q, U, u_off, S, s_off, V, v_off, k_out,
                        stream=None):
    """zs_query_batch into caller-owned device buffers.  t_s, t_e, u_off, s_off,
    v_off: int64 numpy arrays; k_q: int32 numpy array; U, S, V: float64 device
    tensors (offsets in elements); k_out: int32 device tensor of len(t_s)."""
    nq = len(t_s)
    arrs = [np.ascontiguousarray(x, np.int64) for x in (t_s, t_e, u_off, s_off, v_off)]
    kq = np.ascontiguousarray(k_q, np.int32)
    a = lambda x: _vp(x.ctypes.data)
    _check(load().zs_query_batch(_vp(st.handle), nq, a(arrs[0]), a(arrs[1]), a(kq), _vp(_ptr(U)),
                                 a(arrs[2]), _vp(_ptr(S)), a(arrs[3]), _vp(_ptr(V)), a(arrs[4]),
                                 _vp(_ptr(k_out)), _vp(_stream(stream))))


def zs_store_get_block(st: Store, i: int, stream=None):
    """Block i's factors as device tensors: U rows_i x k, S k, V c x k, k_i."""
    dev = torch.device("cuda", torch.cuda.current_device())
    rows = st.block_rows(i)
    U = torch.empty((rows, st.k), dtype=st.out_dtype, device=dev)
    S = torch.empty(st.k, dtype=torch.float64, device=dev)
    V = torch.empty((st.c, st.k), dtype=st.out_dtype, device=dev)
    ki = torch.empty(1, dtype=torch.int32, device=dev)
    _check(load().zs_store_get_block(_vp(st.handle), i, _vp(_ptr(U)), _vp(_ptr(S)), _vp(_ptr(V)),
                                     _vp(_ptr(ki)), _vp(_stream(stream))))
    return U, S, V, ki


def zs_query_scratch_bytes(st: Store, t_s: int, t_e: int, k_q: int) -> int:
    """Device scratch a query adds to its stream's workspace (-1: rejected)."""
    return int(load().zs_query_scratch_bytes(_vp(st.handle), t_s, t_e, k_q))


def zs_store_bytes(st: Store) -> int:
    return int(load().zs_store_bytes(_vp(st.handle)))


def zs_sync_status(st: Store, stream=None):
    _check(load().zs_sync_status(_vp(st.handle), _vp(_stream(stream))))


def zs_release_workspaces(stream=None):
    """Return the scratch the library keeps for a stream (storage phase and
    queries); the next call on the stream allocates again."""
    _check(load().zs_release_workspaces(_vp(_stream(stream))))


def zs_timing_enable(on: bool = True):
    load().zs_timing_enable(1 if on else 0)


def zs_timing_reset():
    load().zs_timing_reset()


def zs_timing_get(name: str):
    """(launches, total_ms) of kernel `name` since the last reset."""
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    _check(load().zs_timing_get(name.encode(), ctypes.byref(n), ctypes.byref(ms)))
    return int(n.value), float(ms.value)


def zs_autotune(on: bool = True):
    """Turns the timing of launch variants on or off (cached choices apply)."""
    load().zs_autotune(1 if on else 0)


def zs_autotune_force(site: str, variant: int):
    """Forces a launch variant at a tuned site for every shape (< 0 clears)."""
    _check(load().zs_autotune_force(site.encode(), variant))


def zs_autotune_table() -> dict:
    """{'site|key': (variant, 'ms,ms')} of the choices made so far."""
    out = {}
    for line in load().zs_autotune_table().decode().splitlines():
        parts = line.split("\t")
        if len(parts) >= 2:
            out[parts[0]] = (int(parts[1]), parts[2] if len(parts) > 2 else "")
    return out


def zs_set_sweep_cap(cap: int):
    """Jacobi sweep cap of the current device (tests of the ZS_ENOCONV path)."""
    _check(load().zs_set_sweep_cap(cap))
