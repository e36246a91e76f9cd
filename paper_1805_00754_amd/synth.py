"""Seeded synthetic inputs: sensor-like multivariate time series and query sets.

This module only draws random numbers; it holds none of Zoom-SVD's
arithmetic.  It is the one piece shared by the GPU path's tests and the CPU
oracle's tests: both are fed the same arrays from here.

The paper's datasets (Activity 382,000 x 41, Gas 4,107,000 x 16, London
350,000 x 10; Sec. 4.1, Table 2) are not available, so these generators stand
in for them with the same shape: tall-skinny matrices whose columns are smooth
periodic sources mixed across sensors, plus noise.

Recipe (all draws from ``numpy.random.Generator(PCG64(seed))``, in this order):
frequencies f_j ~ U[1/2000, 1/20] cycles/row, phases phi_j ~ U[0, 2 pi),
mixing matrix, noise (in row chunks; an AR(1) state is carried across
chunks), then query lengths and starts.  Sources are
s_j(tau) = sin(2 pi f_j tau + phi_j), tau = 0 .. t-1, and A = S @ Mix + noise.
"""
from __future__ import annotations

import dataclasses

import numpy as np

SEED_BASE = 180500754

# Named workloads (rows t, columns c, sources, noise model, block b, rank k).
WORKLOADS = {
    "sinmix_10k_x64_f64": dict(t=10_000, c=64, sources=8, noise="iid", noise_sigma=0.1,
                               dtype="f64", b=100, k=10, seed_offset=1),
    "sinmix_1m_x128_f64": dict(t=1_000_000, c=128, sources=16, noise="ar1", noise_sigma=0.05,
                               ar_phi=0.9, dtype="f64", b=1000, k=20, seed_offset=2),
    "sinmix_4m_x256_f32": dict(t=4_000_000, c=256, sources=32, noise="iid", noise_sigma=0.1,
                               dtype="f32", b=2000, k=32, seed_offset=3),
    "decay_2m_x1024_bf16": dict(t=2_000_000, c=1024, sources=64, noise="iid", noise_sigma=0.01,
                                dtype="bf16", mix="orthonormal", source_decay=0.9, b=4096,
                                k=64, seed_offset=5),
}


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclasses.dataclass
class Series:
    A: np.ndarray            # t x c, float64 (bf16-representable values for "bf16")
    dtype: str               # storage dtype the workload asks for: f64 / f32 / bf16
    rng: np.random.Generator  # continues the draw sequence (queries come next)


def _round_bf16(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), returned as
    float32 holding exactly representable bf16 values."""
    u = np.ascontiguousarray(x, np.float32).view(np.uint32)
    lsb = (u >> 16) & 1
    r = (u + 0x7FFF + lsb) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32)


def sinusoid_mixture(t: int, c: int, sources: int, seed: int, noise: str = "iid",
                     noise_sigma: float = 0.1, ar_phi: float = 0.9, dtype: str = "f64",
                     mix: str = "gauss", source_decay: float | None = None,
                     chunk: int = 1 << 16) -> Series:
    """t x c matrix: `sources` sinusoids mixed into c columns plus noise."""
    rng = rng_for(seed)
    freq = rng.uniform(1.0 / 2000.0, 1.0 / 20.0, size=sources)
    phase = rng.uniform(0.0, 2.0 * np.pi, size=sources)
    if mix == "gauss":
        Mix = rng.standard_normal((sources, c))
    elif mix == "orthonormal":
        G = rng.standard_normal((c, sources))
        Q, R = np.linalg.qr(G)
        Q = Q * np.sign(np.diag(R))[None, :]
        Mix = np.ascontiguousarray(Q.T)
    else:
        raise ValueError(mix)
    if source_decay is not None:
        Mix = Mix * (source_decay ** np.arange(sources))[:, None]
    A = np.empty((t, c), np.float64)
    ar_state = None
    for r0 in range(0, t, chunk):
        r1 = min(t, r0 + chunk)
        tau = np.arange(r0, r1, dtype=np.float64)
        Sblk = np.sin(2.0 * np.pi * tau[:, None] * freq[None, :] + phase[None, :])
        blk = Sblk @ Mix
        if noise == "iid":
            blk += noise_sigma * rng.standard_normal((r1 - r0, c))
        elif noise == "ar1":
            eta = noise_sigma * rng.standard_normal((r1 - r0, c))
            if ar_state is None:
                # stationary start: Var(e) = sigma^2 / (1 - phi^2)
                ar_state = eta[0] / np.sqrt(1.0 - ar_phi * ar_phi)
                e = np.empty_like(eta)
                e[0] = ar_state
                start = 1
            else:
                e = np.empty_like(eta)
                start = 0
            from scipy.signal import lfilter
            if r1 - r0 > start:
                zi = (ar_phi * ar_state)[:, None]
                out, _ = lfilter([1.0], [1.0, -ar_phi], np.ascontiguousarray(eta[start:].T),
                                 axis=-1, zi=zi)
                e[start:] = out.T
            ar_state = e[-1].copy()
            blk += e
        elif noise == "none":
            pass
        else:
            raise ValueError(noise)
        A[r0:r1] = blk
    if dtype == "f32":
        A = A.astype(np.float32).astype(np.float64)
    elif dtype == "bf16":
        A = _round_bf16(A.astype(np.float32)).astype(np.float64)
    return Series(A=A, dtype=dtype, rng=rng)


def workload(name: str, t: int | None = None) -> tuple[Series, dict]:
    """Generate a named workload (optionally with fewer rows, same recipe)."""
    cfg = dict(WORKLOADS[name])
    if t is not None:
        cfg["t"] = t
    seed = SEED_BASE + cfg.pop("seed_offset")
    b, k = cfg.pop("b"), cfg.pop("k")
    ser = sinusoid_mixture(seed=seed, **cfg)
    cfg.update(b=b, k=k, seed=seed)
    return ser, cfg


def queries_uniform(rng: np.random.Generator, t: int, n: int, lmin: int, lmax: int):
    """n ranges with length L ~ U{lmin..lmax} and start ~ U{0..t-L}."""
    L = rng.integers(lmin, lmax + 1, size=n)
    L = np.minimum(L, t)
    ts = np.array([rng.integers(0, t - l + 1) for l in L], np.int64)
    return ts, ts + L


def queries_loguniform(rng: np.random.Generator, t: int, n: int, lmin: float, lmax: float):
    """n ranges with length round(exp(U[ln lmin, ln lmax])) and random start."""
    L = np.rint(np.exp(rng.uniform(np.log(lmin), np.log(lmax), size=n))).astype(np.int64)
    L = np.clip(L, 1, t)
    ts = np.array([rng.integers(0, t - l + 1) for l in L], np.int64)
    return ts, ts + L


def queries_fixed(rng: np.random.Generator, t: int, n: int, length: int):
    """n ranges of exactly `length` rows at random starts."""
    ts = rng.integers(0, t - length + 1, size=n).astype(np.int64)
    return ts, ts + length


def block_low_rank(t: int, c: int, b: int, rank: int, seed: int) -> np.ndarray:
    """Every b-row block has rank exactly `rank` (a fresh random factor pair
    per block); the whole matrix generally has higher rank."""
    rng = rng_for(seed)
    A = np.empty((t, c))
    for r0 in range(0, t, b):
        r1 = min(t, r0 + b)
        L = rng.standard_normal((r1 - r0, rank))
        R = rng.standard_normal((rank, c))
        A[r0:r1] = L @ R
    return A


def rank_one(t: int, c: int, seed: int):
    """A = s m^T with s a sinusoid over time and m a random mixing vector."""
    rng = rng_for(seed)
    f = rng.uniform(1.0 / 2000.0, 1.0 / 20.0)
    ph = rng.uniform(0.0, 2.0 * np.pi)
    s = np.sin(2.0 * np.pi * f * np.arange(t) + ph) + 1.5
    m = rng.standard_normal(c)
    return np.outer(s, m), s, m
