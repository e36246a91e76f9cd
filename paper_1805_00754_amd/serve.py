"""Continuous-batching serving loop over a device-resident store.

Range queries (t_s, t_e, k_q) arrive over time.  The loop keeps the store in
HBM and answers the queries in batches through ``zs_query_batch``:

* admission: a batch takes pending requests first-come first-served while it
  stays within ``max_queries`` and an HBM byte budget per batch: each
  request's outputs (U n x k_q and V c x k_q in the store's output type,
  Sigma k_q in FP64, k_out) plus the device scratch the library adds for it
  (``zs_query_scratch_bytes``); a request that alone exceeds the budget is
  rejected;
* continuous batching: up to ``depth`` batches are in flight, each on its own
  stream (default priority) with its own output arena and its own library
  workspace, so batches overlap on the device while the host plans the next
  one; a new batch is formed as soon as a slot is free and requests wait;
* timing: a HIP event recorded at the start of the run is the time origin,
  and each batch records events when its kernels start and finish, so a
  request's latency is GPU completion time minus its arrival time (open loop:
  arrivals do not wait for completions) and a batch's service time is its
  own device time.

The batch policy is plain host logic (``BatchPolicy``); every query is answered
by the library's kernels.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np


def output_bytes(n: int, kq: int, c: int, esize: int = 8) -> int:
    """Device bytes of one query's outputs: U and V with `esize`-byte elements
    (8 for FP64 stores, 4 for FP32-stored factors), Sigma in FP64, k_out."""
    return esize * (n * kq + c * kq) + 8 * kq + 4


@dataclasses.dataclass
class Request:
    idx: int
    t_s: int
    t_e: int
    k_q: int
    arrival: float          # seconds after the start of the run


class BatchPolicy:
    """First-come first-served packing under a query count and a byte budget.
    A request costs its outputs plus `scratch_fn(request)` bytes (the library's
    device scratch for it; none when not given)."""

    def __init__(self, c: int, max_queries: int, budget_bytes: int, esize: int = 8,
                 scratch_fn=None):
        if max_queries < 1 or budget_bytes < 1:
            raise ValueError("max_queries and budget_bytes must be positive")
        self.c = c
        self.max_queries = max_queries
        self.budget_bytes = budget_bytes
        self.esize = esize
        self.scratch_fn = scratch_fn

    def bytes_of(self, r: Request) -> int:
        out = output_bytes(r.t_e - r.t_s, r.k_q, self.c, self.esize)
        return out + (int(self.scratch_fn(r)) if self.scratch_fn is not None else 0)

    def fits_alone(self, r: Request) -> bool:
        return self.bytes_of(r) <= self.budget_bytes

    def take(self, pending: collections.deque) -> list:
        """Removes and returns the next batch from the head of `pending`."""
        batch, used = [], 0
        while pending and len(batch) < self.max_queries:
            r = pending[0]
            b = self.bytes_of(r)
            if used + b > self.budget_bytes:
                break
            batch.append(pending.popleft())
            used += b
        return batch


def poisson_arrivals(rng: np.random.Generator, rate: float, n: int) -> np.ndarray:
    """n arrival times (seconds) of a Poisson process of the given rate."""
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


class Server:
    """Serves range queries on one store with continuous batching."""

    def __init__(self, st, max_queries: int = 256, budget_bytes: int = 1 << 30, depth: int = 2):
        import torch

        from . import zoomsvd as zs

        self.zs = zs
        self.torch = torch
        self.st = st
        esize = torch.empty((), dtype=st.out_dtype).element_size()
        self.policy = BatchPolicy(st.c, max_queries, budget_bytes, esize,
                                  scratch_fn=lambda r: zs.zs_query_scratch_bytes(st, r.t_s, r.t_e,
                                                                                  r.k_q))
        self.depth = depth
        # one stream per in-flight slot, all at the default priority
        self.streams = [torch.cuda.Stream() for _ in range(depth)]
        self.stream = torch.cuda.current_stream()          # the time origin's stream
        dev = torch.device("cuda", torch.cuda.current_device())
        # one output arena per in-flight slot: U and V share a flat buffer of the
        # store's output type, Sigma has an FP64 one
        self.arena = [torch.empty(budget_bytes // esize, dtype=st.out_dtype, device=dev)
                      for _ in range(depth)]
        self.sarena = [torch.empty(max_queries * st.k, dtype=torch.float64, device=dev)
                       for _ in range(depth)]
        self.kout = [torch.empty(max_queries, dtype=torch.int32, device=dev) for _ in range(depth)]

    def _launch(self, slot: int, batch: list):
        c = self.st.c
        n = np.array([r.t_e - r.t_s for r in batch], np.int64)
        kq = np.array([r.k_q for r in batch], np.int32)
        sizes_u = n * kq
        u_off = np.zeros(len(batch), np.int64)
        u_off[1:] = np.cumsum(sizes_u)[:-1]
        s_off = np.concatenate(([0], np.cumsum(kq)[:-1])).astype(np.int64)
        v_base = int(sizes_u.sum())
        v_off = v_base + np.concatenate(([0], np.cumsum(c * kq.astype(np.int64))[:-1])).astype(np.int64)
        a = self.arena[slot]
        stream = self.streams[slot]
        start = self.torch.cuda.Event(enable_timing=True)
        start.record(stream)
        self.zs.zs_query_batch_into(self.st, [r.t_s for r in batch], [r.t_e for r in batch], kq,
                                    a, u_off, self.sarena[slot], s_off, a, v_off, self.kout[slot],
                                    stream=stream)
        done = self.torch.cuda.Event(enable_timing=True)
        done.record(stream)
        return dict(slot=slot, batch=batch, start=start, done=done, u_off=u_off, s_off=s_off,
                    v_off=v_off)

    def run(self, requests: list, on_batch=None) -> dict:
        """Serves `requests` (sorted by arrival) in real time.  Returns per-request
        completion times and latencies (seconds) and batch statistics.
        `on_batch(info, arena, sarena, kout)` is called after a batch completes
        (tests): U and V of the batch are in `arena`, Sigma in `sarena`."""
        torch = self.torch
        n = len(requests)
        completion = np.full(n, np.nan)
        rejected = []
        pending = collections.deque()
        inflight = collections.deque()
        free = list(range(self.depth))
        batches = []
        torch.cuda.synchronize()
        origin = torch.cuda.Event(enable_timing=True)
        origin.record(self.stream)
        origin.synchronize()
        t0 = time.perf_counter()
        nxt = 0
        finished = 0

        batch_ms = []

        def retire(info):
            nonlocal finished
            info["done"].synchronize()
            t_done = origin.elapsed_time(info["done"]) / 1e3
            batch_ms.append(info["start"].elapsed_time(info["done"]))
            for r in info["batch"]:
                completion[r.idx] = t_done
            finished += len(info["batch"])
            if on_batch is not None:
                on_batch(info, self.arena[info["slot"]], self.sarena[info["slot"]],
                         self.kout[info["slot"]])
            free.append(info["slot"])

        while finished + len(rejected) < n:
            now = time.perf_counter() - t0
            while nxt < n and requests[nxt].arrival <= now:
                r = requests[nxt]
                if self.policy.fits_alone(r):
                    pending.append(r)
                else:
                    rejected.append(r.idx)
                nxt += 1
            while inflight and inflight[0]["done"].query():
                retire(inflight.popleft())
            if pending and free:
                batch = self.policy.take(pending)
                info = self._launch(free.pop(0), batch)
                inflight.append(info)
                batches.append(len(batch))
                continue
            if not pending and nxt < n:
                wait = requests[nxt].arrival - (time.perf_counter() - t0)
                if wait > 2e-4:
                    time.sleep(min(wait, 1e-3) - 1e-4)
            elif inflight and not free:
                retire(inflight.popleft())
        while inflight:
            retire(inflight.popleft())
        arrival = np.array([r.arrival for r in requests])
        lat = completion - arrival
        ok = ~np.isnan(lat)
        return dict(completion=completion, latency=lat, rejected=rejected, batches=batches,
                    batch_ms=batch_ms,
                    p50=float(np.percentile(lat[ok], 50)) if ok.any() else None,
                    p99=float(np.percentile(lat[ok], 99)) if ok.any() else None,
                    span=float(np.nanmax(completion)) if ok.any() else 0.0)


def fifo_replay(arrival: np.ndarray, service: np.ndarray) -> np.ndarray:
    """Completion times of requests served one at a time in arrival order
    (a single server, first-come first-served) with the given service times:
    each starts when it has arrived and the previous one has finished."""
    done = np.empty(len(arrival))
    t = 0.0
    for i in range(len(arrival)):
        t = max(t, float(arrival[i])) + float(service[i])
        done[i] = t
    return done


def make_requests(rng: np.random.Generator, t: int, n: int, rate: float, lmin: float, lmax: float,
                  kq_choices) -> list:
    """n requests: Poisson arrivals, log-uniform lengths in [lmin, lmax], random
    starts, k_q uniform over `kq_choices`."""
    arr = poisson_arrivals(rng, rate, n)
    L = np.rint(np.exp(rng.uniform(np.log(lmin), np.log(lmax), size=n))).astype(np.int64)
    L = np.clip(L, 1, t)
    ts = np.array([rng.integers(0, t - l + 1) for l in L], np.int64)
    kq = rng.choice(np.asarray(kq_choices, np.int32), size=n)
    return [Request(i, int(ts[i]), int(ts[i] + L[i]), int(kq[i]), float(arr[i])) for i in range(n)]
