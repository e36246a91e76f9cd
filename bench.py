"""Benchmark of the Zoom-SVD hot path on one MI355X.

One step = the whole hot path over one batch of synthetic input:
  storage phase  zs_store_blocks  on A (1,000,000 x 128 float64, b = 1000, k = 20)
  query phase    zs_query_batch   on 1,024 ranges of exactly 320,000 rows, k_q = 20.
Inputs are resident in HBM before the timed region starts.

Printed as one JSON line:
  value       range-query SVDs/s of the batched query phase (1,024 / query time)
  p50/p99     latency of single queries (zs_query, one at a time) of 320,000 rows
  store_gbps  storage-phase throughput, t * c * 8 bytes / store time
  roofline    the dominant kernel against its roofline (HIP events on the
              library's stream, over the timed steps)
  cpu_baseline the CPU oracle timed on a bounded sample of the same workload
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "sinmix_1m_x128_f64"
QUERY_LEN = 320_000
N_QUERIES = 1024
# The query batch of each workload: (distribution, queries, range lengths).
# fixed: every range QUERY_LEN rows; loguniform: lengths log-uniform in [lo, hi]
# at random starts (uneven stacks of whole blocks plus partial boundaries).
BATCHES = {
    "sinmix_10k_x64_f64": ("uniform", 20, 150, 8_000),
    "sinmix_1m_x128_f64": ("fixed", N_QUERIES, QUERY_LEN, QUERY_LEN),
    "sinmix_4m_x256_f32": ("loguniform", 1024, 10_000, 320_000),
    "decay_2m_x1024_bf16": ("loguniform", 512, 100_000, 1_000_000),
}
HBM_PEAK_GBPS = 8000.0
FP64_PEAK_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--queries", type=int, default=None,
                    help="queries per batch (default: the workload's batch)")
    ap.add_argument("--query-dist", default=None, choices=["fixed", "loguniform", "uniform"],
                    help="range lengths of the batch (default: the workload's batch)")
    ap.add_argument("--latency-samples", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-queries", type=int, default=32)
    ap.add_argument("--serve-rates", default=None,
                    help="arrival rates (queries/s) of the serving runs; empty to skip "
                         "(default 500,2000,8000 on the default workload, none on others)")
    ap.add_argument("--serve-requests", type=int, default=3000)
    ap.add_argument("--serve-single", type=int, default=128,
                    help="sample of one-at-a-time FP64 queries timed for the serving baseline")
    ap.add_argument("--workload", default=WORKLOAD,
                    help="named synthetic workload (synth.WORKLOADS); the default is the one "
                         "the headline metric is quoted on")
    ap.add_argument("--query-len", type=int, default=QUERY_LEN,
                    help="range length of a fixed batch")
    ap.add_argument("--sweep-queries", type=int, default=256,
                    help="queries per batch of the block-size study in the default run "
                         "(0 skips it)")
    ap.add_argument("--sweep-b", default=None,
                    help="comma-separated block sizes: instead of the benchmark, store the "
                         "workload at each b and time query batches at range lengths 1e3, 1e4 "
                         "and 1e5 (the paper's block-size study), one JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1805_00754_amd import synth
    from paper_1805_00754_amd import zoomsvd as zs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    zs.load()
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()

    if args.sweep_b:
        return sweep_b(args)

    wl = args.workload
    log("generating %s" % wl)
    ser, cfg = synth.workload(wl)
    A_host = ser.A
    t, c = A_host.shape
    b, k = cfg["b"], cfg["k"]
    tdtype, mode, esize = {"f64": (torch.float64, zs.ZS_MODE_FP64, 8),
                           "f32": (torch.float32, zs.ZS_MODE_FP32, 4),
                           "bf16": (torch.bfloat16, zs.ZS_MODE_BF16, 2)}[cfg["dtype"]]
    usize = 8 if mode == zs.ZS_MODE_FP64 else 4       # stored U / V element size
    dist, nq_default, lmin, lmax = BATCHES.get(wl, ("fixed", N_QUERIES, QUERY_LEN, QUERY_LEN))
    dist = args.query_dist or dist
    if args.queries is None:
        args.queries = nq_default
    if dist == "fixed":
        qlen = min(args.query_len, t)
        ts, te = synth.queries_fixed(ser.rng, t, args.queries, qlen)
        batch_desc = "%d ranges of %d rows" % (args.queries, qlen)
    elif dist == "loguniform":
        ts, te = synth.queries_loguniform(ser.rng, t, args.queries, lmin, min(lmax, t))
        qlen = int(np.median(te - ts))
        batch_desc = "%d ranges, lengths log-uniform in [%g, %g] rows" % (args.queries, lmin, lmax)
    else:
        ts, te = synth.queries_uniform(ser.rng, t, args.queries, lmin, min(lmax, t))
        qlen = int(np.median(te - ts))
        batch_desc = "%d ranges, lengths uniform in [%d, %d] rows" % (args.queries, lmin, lmax)
    kq = np.full(args.queries, k, np.int32)
    A = torch.from_numpy(A_host).to(dev).to(tdtype)
    torch.cuda.synchronize()

    # Output buffers of the batch are allocated once, outside the timed region.
    st0 = zs.zs_store_blocks(A, b, k, mode=mode)
    out = zs.Batch(st0, ts, te, kq, dev)
    st0.free()

    def step(timing_events=None):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e2 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        st = zs.zs_store_blocks(A, b, k, mode=mode)   # synchronises the stream at its end
        e1.record(stream)
        zs.zs_query_batch(st, ts, te, kq, out=out)
        e2.record(stream)
        e2.synchronize()
        return st, e0.elapsed_time(e1), e1.elapsed_time(e2)

    log("warmup %d" % args.warmup)
    for _ in range(args.warmup):
        st, _, _ = step()
        zs.zs_sync_status(st)
        st.free()

    zs.zs_timing_reset()
    zs.zs_timing_enable(True)
    torch.cuda.synchronize()
    store_ms, query_ms = [], []
    t0 = time.perf_counter()
    for i in range(args.steps):
        st, sm, qm = step()
        store_ms.append(sm)
        query_ms.append(qm)
        if i + 1 < args.steps:
            st.free()
        log("step %d: store %.2f ms  query batch %.2f ms" % (i, sm, qm))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    zs.zs_timing_enable(False)
    kernels = {}
    for name in ("gram", "eig", "project", "finalize", "utransform", "leaf_gram", "tree_level",
                 "expand", "order", "partial", "stack_project", "coef", "blockprod"):
        n, ms = zs.zs_timing_get(name)
        if n:
            kernels[name] = {"launches": n, "total_ms": ms, "avg_ms": ms / n}
    zs.zs_sync_status(st)

    # The same batch replayed from a captured HIP graph: no host planning or
    # descriptor upload inside the timed replays.
    g = zs.zs_query_batch_graph(st, ts, te, kq, out=out)
    torch.cuda.synchronize()
    graph_ms = []
    for _ in range(3):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        g.launch(stream)
        e1.record(stream)
        e1.synchronize()
        graph_ms.append(e0.elapsed_time(e1))
    g.free()
    log("graph replay %.2f ms" % float(np.mean(graph_ms)))

    # The storage phase captured into a graph (zs_store_graph_create) and
    # replayed on the same input: one graph launch per store, no host
    # planning, allocation or synchronisation inside it.
    sg = zs.zs_store_graph_create(A, b, k, mode=mode)
    torch.cuda.synchronize()
    gstore_ms = []
    for _ in range(3):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sg.launch(stream)
        e1.record(stream)
        e1.synchronize()
        gstore_ms.append(e0.elapsed_time(e1))
    zs.zs_sync_status(sg.st)
    sg.free()
    sg.st.free()
    log("store graph replay %.2f ms" % float(np.mean(gstore_ms)))

    # The case study of Sec. 5: u_1 of every earlier 20,000-row window (stride
    # 500) against u_1 of the last 20,000 rows, all windows as one batch.
    windows = None
    if wl == WORKLOAD and t >= 40_000:
        W, stride = 20_000, 500
        base = t - W
        nw = base // stride
        sim = zs.zs_window_similarity(st, base, t, stride, nw)      # warm-up
        torch.cuda.synchronize()
        wms = []
        for _ in range(3):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            zs.zs_window_similarity(st, base, t, stride, nw, sim=sim)
            e1.record(stream)
            e1.synchronize()
            wms.append(e0.elapsed_time(e1))
        top = torch.topk(sim, 2).indices.cpu().numpy() + 1
        windows = {"window_rows": W, "stride": stride, "windows": nw,
                   "ms": float(np.mean(wms)), "windows_per_s": nw / (float(np.mean(wms)) / 1e3),
                   "most_similar_offsets_rows": [int(x) * stride for x in top]}
        log("window similarity: %d windows in %.2f ms" % (nw, windows["ms"]))

    # Streaming ingest: ten appends of 1,000 rows each (one block's worth, cut
    # across block boundaries) to a copy of the benchmark store.
    ingest = None
    if wl == WORKLOAD:
        extra = synth.sinusoid_mixture(11_000, c, sources=16, seed=synth.SEED_BASE + 11,
                                       noise="ar1", noise_sigma=0.05).A
        R = torch.from_numpy(extra).to(dev)
        sa = zs.zs_store_blocks(A[:t - 500], b, k, mode=mode)     # last block half full
        zs.zs_store_append(sa, R[:1_000])                          # warm-up
        torch.cuda.synchronize()
        ams = []
        for j in range(1, 11):
            a0 = time.perf_counter()
            zs.zs_store_append(sa, R[j * 1_000:(j + 1) * 1_000])
            ams.append((time.perf_counter() - a0) * 1e3)
        sa.free()
        ingest = {"rows_per_append": 1_000, "appends": 10, "ms_per_append": float(np.median(ams)),
                  "rows_per_s": 1_000 / (float(np.median(ams)) / 1e3), "store_rows": t - 500}
        log("ingest: %.2f ms per 1,000-row append" % ingest["ms_per_append"])

    # Write ceiling of this very output allocation: a plain fill of the batch's
    # U buffer.  Sustained write bandwidth into a large allocation depends on
    # where it landed in physical memory (5.5 to 6.9 TB/s seen for the same
    # 52 GB size), so blockprod is also measured against this figure.
    # Two plain writers, torch's fill and zeroing (a runtime memset); the faster
    # one's mean over three passes is the ceiling.
    fills = {}
    for name, fn in (("fill", lambda: out.U.fill_(1.0)), ("zero", lambda: out.U.zero_())):
        ms = []
        for _ in range(3):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        fills[name] = float(np.mean(ms))
    fill_ms = min(fills.values())
    out_bytes = out.U.numel() * out.U.element_size()
    fill_gbps = out_bytes / (fill_ms / 1e3) / 1e9
    log("writers of the output buffer: %s; ceiling %.0f GB/s"
        % (", ".join("%s %.2f ms" % kv for kv in fills.items()), fill_gbps))

    # Single-query latency (queries issued one at a time).
    lat = []
    U1 = torch.empty((int((te - ts).max()), k), dtype=st.out_dtype, device=dev)
    S1 = torch.empty(k, dtype=torch.float64, device=dev)
    V1 = torch.empty((c, k), dtype=st.out_dtype, device=dev)
    ko = torch.empty(1, dtype=torch.int32, device=dev)
    for q in range(min(args.latency_samples + 4, args.queries)):
        torch.cuda.synchronize()
        a = time.perf_counter()
        zs.zs_query(st, int(ts[q]), int(te[q]), k, U1, S1, V1, ko)
        torch.cuda.synchronize()
        if q >= 4:
            lat.append((time.perf_counter() - a) * 1e3)
    if args.serve_rates is None:
        args.serve_rates = "500,2000,8000" if wl == WORKLOAD else ""
    serving = serve_runs(st, args, A, b, k, mode) if args.serve_rates else None
    # The block-size study of Sec. 4.5 on the benchmark series (b = 10 to 10^5).
    sweep = None
    if wl == WORKLOAD and args.sweep_queries > 0:
        sweep = block_size_sweep(A, k, [10, 100, 1_000, 10_000, 100_000], args.sweep_queries)
    # Reduced-precision modes: every query of the batch against the FP64 path
    # (an FP64-mode store of the same input, the same batch), per result.
    precision = None
    if mode != zs.ZS_MODE_FP64:
        precision = precision_vs_fp64(A, b, k, st, ts, te, kq, out, dev)
    st.free()

    q_ms = float(np.mean(query_ms))
    s_ms = float(np.mean(store_ms))
    value = args.queries / (q_ms / 1e3)
    store_gbps = t * c * esize / (s_ms / 1e3) / 1e9

    # Roofline of the dominant kernel (largest share of the timed region).
    n_rows = int((te - ts).sum())
    pieces = int(sum((int(e) - 1) // b - int(s) // b + 1 for s, e in zip(ts, te)))
    kp = prod_ld(k)
    algo = {
        # per query: its U rows read (k values each) and written (k_q each), plus
        # one k x k_q coefficient block per touched block (stored k_q x prod_ld(k))
        "blockprod": ("hbm", usize * 2.0 * n_rows * k + 8.0 * pieces * kp * k, "GB/s"),
        # A read once
        "gram": ("hbm", esize * t * c, "GB/s"),
        "project": ("hbm", esize * t * c + 8.0 * t * k, "GB/s"),
    }
    # Bytes the batched block product must move across HBM at least once: the
    # stored U rows its queries touch (each once, however many queries read
    # it), one coefficient block per piece, and the output rows.
    touched = np.zeros(t, bool)
    for s_, e_ in zip(ts, te):
        touched[int(s_):int(e_)] = True
    u_rows = int(touched.sum())
    unique_bp = usize * (u_rows * k + n_rows * k) + 8.0 * pieces * kp * k
    dom = max(kernels, key=lambda n: kernels[n]["total_ms"])
    if dom in algo:
        bound, amount, unit = algo[dom]
        avg_s = kernels[dom]["avg_ms"] / 1e3
        if dom == "blockprod":
            amount_hbm = unique_bp
        else:
            amount_hbm = amount
        achieved = amount_hbm / avg_s / 1e9
        roof = {"kernel": dom, "bound": bound, "achieved": achieved, "peak": HBM_PEAK_GBPS,
                "unit": unit, "frac": achieved / HBM_PEAK_GBPS,
                "traffic": profiled_traffic(dom, wl), "algorithmic_bytes_per_launch": amount_hbm,
                "avg_launch_ms": avg_s * 1e3}
        if dom == "blockprod":
            # Per-query accounting: every query reads its own U rows, so rows
            # shared by overlapping ranges count once per query.  Those repeat
            # reads are served from L2 (block-major order), which is why this
            # figure exceeds the HBM peak; it is not an HBM fraction.
            roof["per_query_bytes_per_launch"] = amount
            roof["per_query_rate_gbps"] = amount / avg_s / 1e9
            # the output alone against a plain fill of the same allocation
            roof["output_write_gbps"] = out_bytes / avg_s / 1e9
            roof["fill_gbps_same_buffer"] = fill_gbps
            roof["output_frac_of_fill"] = out_bytes / avg_s / 1e9 / fill_gbps
    elif dom == "eig":
        # FP64 arithmetic of the eigen-solves: one c x c problem per block and
        # per query, (4/3) c^3 flops of tridiagonalisation and 2 c^2 k of
        # back-transformation each
        n_eig = kernels["eig"]["launches"] / args.steps
        flops = ((t + b - 1) // b + args.queries) * (4.0 / 3.0 * c ** 3 + 2.0 * c * c * k)
        sec = kernels["eig"]["total_ms"] / args.steps / 1e3
        roof = {"kernel": "eig", "bound": "fp64", "achieved": flops / sec / 1e12,
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": flops / sec / 1e12 / FP64_PEAK_TFLOPS, "traffic": None,
                "algorithmic_flops_per_step": flops, "launches_per_step": n_eig,
                "ms_per_step": sec * 1e3}
    else:
        roof = {"kernel": dom, "bound": "alu", "achieved": None, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": None, "traffic": None}

    # Every timed kernel against its own binding roof, per step (store + batch).
    # Units of work: the store's t rows, nb blocks (one c x c eigen-problem
    # each, with k kept), and the batch's queries (one c x c eigen-problem each),
    # pieces and boundary blocks.  Flops count what the method must do; bytes
    # count each operand once.
    nb = (t + b - 1) // b
    nq = args.queries
    part_rows = 0                     # rows of the boundary blocks cut by the ranges
    for s_, e_ in zip(ts, te):
        s_, e_ = int(s_), int(e_)
        S_, E_ = s_ // b, (e_ - 1) // b
        if S_ == E_:
            part_rows += (e_ - s_) if (s_ % b or e_ - S_ * b != min(b, t - S_ * b)) else 0
            continue
        part_rows += (min(b, t - S_ * b) - (s_ - S_ * b)) if s_ % b else 0
        part_rows += (e_ - E_ * b) if e_ - E_ * b != min(b, t - E_ * b) else 0
    eig_flops = (nb + nq) * (4.0 / 3.0 * c ** 3 + 2.0 * c * c * k)
    per_kernel = {
        "gram": ("mfma_fp64", float(t) * c * (c + 1), FP64_PEAK_TFLOPS),
        "project": ("hbm", esize * t * c + 8.0 * t * k, HBM_PEAK_GBPS),
        "utransform": ("hbm", 16.0 * t * k, HBM_PEAK_GBPS),
        "eig": ("fp64", eig_flops, FP64_PEAK_TFLOPS),
        "partial": ("hbm", usize * part_rows * k, HBM_PEAK_GBPS),
        "stack_project": ("mfma_fp64", 2.0 * pieces * k * c * k, FP64_PEAK_TFLOPS),
        "coef": ("hbm", 8.0 * pieces * (k * k + kp * k), HBM_PEAK_GBPS),
        "blockprod": ("hbm", unique_bp, HBM_PEAK_GBPS),
    }
    kernel_roofs = {}
    for name, (bound, amount, peak) in per_kernel.items():
        if name not in kernels:
            continue
        sec = kernels[name]["total_ms"] / args.steps / 1e3
        if bound == "hbm":
            ach = amount / sec / 1e9
            kernel_roofs[name] = {"bound": "hbm", "achieved": ach, "peak": peak, "unit": "GB/s",
                                  "frac": ach / peak, "ms_per_step": sec * 1e3}
        else:
            ach = amount / sec / 1e12
            kernel_roofs[name] = {"bound": bound, "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                                  "frac": ach / peak, "ms_per_step": sec * 1e3}

    cpu = None
    if not args.no_cpu_baseline and wl == WORKLOAD:
        cpu = cpu_baseline(A_host, b, k, ts, te, args.cpu_queries)

    res = {
        "metric": "range-query SVDs/s + p50/p99 latency at 3.2e5-row ranges; store-phase GB/s",
        "value": value,
        "unit": "SVDs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "storage": "f64" if usize == 8 else "f32",
        "data": "synthetic",
        "config": {"workload": wl, "t": t, "c": c, "b": b, "k": k, "input": cfg["dtype"],
                   "queries": args.queries, "query_rows": qlen, "batch": batch_desc,
                   "batch_rows": int((te - ts).sum()), "k_q": k, "parallelism": "single-gpu"},
        "query_batch_ms": q_ms,
        "graph_batch_ms": float(np.mean(graph_ms)),
        "graph_svds_per_s": args.queries / (float(np.mean(graph_ms)) / 1e3),
        "store_ms": s_ms,
        "store_gbps": store_gbps,
        "graph_store_ms": float(np.mean(gstore_ms)),
        "graph_store_gbps": t * c * esize / (float(np.mean(gstore_ms)) / 1e3) / 1e9,
        "store_frac_hbm": store_gbps / HBM_PEAK_GBPS,
        "p50_ms": float(np.percentile(lat, 50)) if lat else None,
        "p99_ms": float(np.percentile(lat, 99)) if lat else None,
        "single_query_svds_per_s": 1e3 / float(np.mean(lat)) if lat else None,
        "kernels_ms_per_step": {n: v["total_ms"] / args.steps for n, v in kernels.items()},
        "roofline": roof,
        "kernel_rooflines": kernel_roofs,
        "serving": serving,
        "windows": windows,
        "ingest": ingest,
        "precision_vs_fp64": precision,
        "block_size_sweep": sweep,
        "autotune": {k_: {"variant": v[0], "ms": v[1]} for k_, v in zs.zs_autotune_table().items()},
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


def precision_vs_fp64(A, b, k, st, ts, te, kq, out, dev, chunk=64):
    """Error of each result of a reduced-precision store against the FP64 path
    on the same input: the FP64-mode store of A answers the same queries
    (in chunks of `chunk`, so that its FP64 outputs stay small).  Per query:
    the largest relative error over sigma_1..k_out (|error| / sigma_1 below
    10 sqrt(c) 6e-8 sigma_1) and the sine of the largest principal angle
    between the two V (leading k_out columns)."""
    import numpy as np
    import torch

    from paper_1805_00754_amd import zoomsvd as zs

    c = st.c
    floor = 10.0 * np.sqrt(c) * 6e-8
    st64 = zs.zs_store_blocks(A, b, k, mode=zs.ZS_MODE_FP64)
    torch.cuda.synchronize()
    sig, ang, kdiff = [], [], 0
    for q0 in range(0, len(ts), chunk):
        q1 = min(len(ts), q0 + chunk)
        ref = zs.zs_query_batch(st64, ts[q0:q1], te[q0:q1], kq[q0:q1])
        torch.cuda.synchronize()
        for q in range(q0, q1):
            _, S, V, ko = out.result(q)
            _, S64, V64, ko64 = ref.result(q - q0)
            S, S64 = S.cpu().numpy(), S64.cpu().numpy()
            kk = int(ko.item())
            kdiff += kk != int(ko64.item())
            kk = min(kk, int(ko64.item()))
            s1 = max(S64[0], 1e-300)
            rel = [abs(S[j] - S64[j]) / (S64[j] if S64[j] > floor * s1 else s1) for j in range(kk)]
            sig.append(max(rel) if rel else 0.0)
            Va = V[:, :kk].double().cpu().numpy()
            Vb = V64[:, :kk].cpu().numpy()
            sv = np.linalg.svd(Va.T @ Vb, compute_uv=False) if kk else np.ones(1)
            ang.append(float(np.sqrt(max(0.0, 1.0 - min(1.0, sv.min()) ** 2))))
        del ref
    st64.free()
    sig, ang = np.array(sig), np.array(ang)
    log("precision vs FP64: sigma rel max %.3g p50 %.3g; V angle max %.3g"
        % (sig.max(), np.median(sig), ang.max()))
    return {"reference": "FP64-mode store of the same input, same queries",
            "sigma_rel_max": float(sig.max()), "sigma_rel_p50": float(np.median(sig)),
            "sigma_rel_p99": float(np.percentile(sig, 99)),
            "v_sin_angle_max": float(ang.max()), "v_sin_angle_p50": float(np.median(ang)),
            "k_out_differs": int(kdiff),
            "per_query_sigma_rel": [float("%.3g" % x) for x in sig]}


def block_size_sweep(A, k, bs, nq, lengths=(1_000, 10_000, 100_000)):
    """The paper's block-size study (Sec. 4.5, Fig. 6) on the device series A:
    for each b, the store time, the stored elements against the raw matrix
    (Thm. 3: sum_i k_i (b_i + 1 + c), k_i = min(k, b_i) on these full-rank
    noisy blocks) and the time of a batch of nq queries at each range length
    (medians of three after one untimed run)."""
    import numpy as np
    import torch

    from paper_1805_00754_amd import synth
    from paper_1805_00754_amd import zoomsvd as zs

    dev = A.device
    stream = torch.cuda.current_stream()
    t, c = A.shape

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            ms.append(e0.elapsed_time(e1))
        return float(np.median(ms))

    rows = []
    for b in bs:
        log("block-size sweep: b = %d" % b)
        holder = {}

        def store():
            if "st" in holder:
                holder.pop("st").free()
            holder["st"] = zs.zs_store_blocks(A, b, k)
        store_ms = timed(store)
        st = holder["st"]
        nb = (t + b - 1) // b
        brows = np.minimum(b, t - np.arange(nb) * b)
        elems = int((np.minimum(k, brows) * (brows + 1 + c)).sum())
        q = {}
        for L in lengths:
            ts, te = synth.queries_fixed(synth.rng_for(synth.SEED_BASE + 9), t, nq, L)
            out = zs.Batch(st, ts, te, np.full(nq, k, np.int32), dev)
            qms = timed(lambda: zs.zs_query_batch(st, ts, te, k, out=out))
            q[str(L)] = {"batch_ms": qms, "svds_per_s": nq / (qms / 1e3)}
            del out
        rows.append({"b": b, "blocks": nb, "store_ms": store_ms,
                     "store_gbps": t * c * A.element_size() / (store_ms / 1e3) / 1e9,
                     "stored_elements": elems, "compression": t * c / elems,
                     "store_bytes": zs.zs_store_bytes(st), "queries": q})
        st.free()
        torch.cuda.empty_cache()
    return {"workload_rows": t, "c": c, "k": k, "queries_per_batch": nq,
            "range_lengths": list(lengths), "sweep": rows}


def sweep_b(args):
    """--sweep-b: the block-size study alone, one JSON line."""
    import torch

    from paper_1805_00754_amd import synth
    from paper_1805_00754_amd import zoomsvd as zs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    zs.load()
    ser, cfg = synth.workload(args.workload)
    A = torch.from_numpy(ser.A).to(torch.device("cuda", 0))
    res = block_size_sweep(A, cfg["k"], [int(x) for x in args.sweep_b.split(",") if x],
                           args.queries or N_QUERIES)
    res.update(metric="block-size sweep (store time, compression, query batches)",
               workload=args.workload)
    print(json.dumps(res), flush=True)


def serve_runs(st, args, A, b, k, mode):
    """Open-loop serving on the resident store: Poisson arrivals at each rate,
    lengths log-uniform in [1e4, 3.2e5] rows, k_q uniform over {8, 16, k};
    two batches in flight on two streams.  Beside it, one-at-a-time FP64
    queries (an FP64-mode store of the same input): their service times are
    measured on the GPU for a sample of the stream's queries, and the stream
    is replayed through a single first-come first-served server with those
    times (the service time of a request: the measured query of the nearest
    length)."""
    import numpy as np
    import torch

    from paper_1805_00754_amd import serve, synth
    from paper_1805_00754_amd import zoomsvd as zs

    dev = torch.device("cuda", 0)
    # one-at-a-time FP64 service times
    st64 = st if mode == zs.ZS_MODE_FP64 else zs.zs_store_blocks(A, b, k, mode=zs.ZS_MODE_FP64)
    rng = synth.rng_for(synth.SEED_BASE + 4)
    sample = serve.make_requests(rng, st.t, args.serve_single, 1.0, 1e4, 3.2e5, [8, 16, st.k])
    nmax = max(r.t_e - r.t_s for r in sample)
    U1 = torch.empty((nmax, st.k), dtype=torch.float64, device=dev)
    S1 = torch.empty(st.k, dtype=torch.float64, device=dev)
    V1 = torch.empty((st.c, st.k), dtype=torch.float64, device=dev)
    ko = torch.empty(1, dtype=torch.int32, device=dev)
    for r in sample[:4]:                                   # warm-up
        zs.zs_query(st64, r.t_s, r.t_e, r.k_q, U1[:, :r.k_q], S1[:r.k_q], V1[:, :r.k_q], ko)
    svc_len, svc_s = [], []
    for r in sample:
        torch.cuda.synchronize()
        a = time.perf_counter()
        zs.zs_query(st64, r.t_s, r.t_e, r.k_q, U1[:, :r.k_q], S1[:r.k_q], V1[:, :r.k_q], ko)
        torch.cuda.synchronize()
        svc_s.append(time.perf_counter() - a)
        svc_len.append(r.t_e - r.t_s)
    if st64 is not st:
        st64.free()
    order = np.argsort(svc_len)
    svc_len = np.asarray(svc_len)[order]
    svc_s = np.asarray(svc_s)[order]
    single = {"store": "fp64", "sample": len(sample), "p50_ms": float(np.median(svc_s) * 1e3),
              "p99_ms": float(np.percentile(svc_s, 99) * 1e3),
              "capacity_per_s": float(1.0 / np.mean(svc_s))}
    log("one-at-a-time FP64: p50 %.2f ms, capacity %.0f queries/s"
        % (single["p50_ms"], single["capacity_per_s"]))

    out = []
    for rate in [float(x) for x in args.serve_rates.split(",") if x]:
        rng = synth.rng_for(synth.SEED_BASE + 4)
        reqs = serve.make_requests(rng, st.t, args.serve_requests, rate, 1e4, 3.2e5,
                                   [8, 16, st.k])
        srv = serve.Server(st, max_queries=512, budget_bytes=4 << 30, depth=2)
        log("serving %d requests at %g/s" % (len(reqs), rate))
        res = srv.run(reqs)
        served = len(reqs) - len(res["rejected"])
        # the same stream served one query at a time in FP64
        L = np.array([r.t_e - r.t_s for r in reqs])
        idx = np.clip(np.searchsorted(svc_len, L), 0, len(svc_len) - 1)
        idx0 = np.clip(idx - 1, 0, len(svc_len) - 1)
        near = np.where(np.abs(svc_len[idx0] - L) < np.abs(svc_len[idx] - L), idx0, idx)
        arr = np.array([r.arrival for r in reqs])
        done = serve.fifo_replay(arr, svc_s[near])
        lat1 = done - arr
        out.append({"rate_per_s": rate, "requests": len(reqs), "served": served,
                    "p50_ms": res["p50"] * 1e3, "p99_ms": res["p99"] * 1e3,
                    "throughput_per_s": served / res["span"],
                    "batches": len(res["batches"]),
                    "mean_batch": float(np.mean(res["batches"])),
                    "batch_p50_ms": float(np.median(res["batch_ms"])),
                    "batch_p99_ms": float(np.percentile(res["batch_ms"], 99)),
                    "one_at_a_time_fp64": {"p50_ms": float(np.median(lat1) * 1e3),
                                           "p99_ms": float(np.percentile(lat1, 99) * 1e3),
                                           "throughput_per_s": len(reqs) / float(done[-1])}})
        log("  p50 %.2f ms p99 %.2f ms (one at a time FP64: p50 %.1f ms p99 %.1f ms)"
            % (out[-1]["p50_ms"], out[-1]["p99_ms"], out[-1]["one_at_a_time_fp64"]["p50_ms"],
               out[-1]["one_at_a_time_fp64"]["p99_ms"]))
        del srv
    return {"single_fp64": single, "rates": out}


def prod_ld(k):
    """Row stride of a stored coefficient block (k rounded up to a compiled width)."""
    return (k + 3) & ~3 if k <= 32 else (k + 15) & ~15


def profiled_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary of this
    kernel on this workload (FETCH_SIZE and WRITE_SIZE scaled by a plain copy),
    or None when there is none or the kernel source has changed since."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "%s_%s.md" % (kernel, workload))
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line:
            key, _, val = line.strip().partition(":")
            fields[key.strip()] = val.strip()
    try:
        src = os.path.join(ROOT, fields["source"])
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if sha != fields["source_sha256"]:
            return None
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, OSError, ValueError):
        return None


def cpu_baseline(A, b, k, ts, te, nq, n_direct=8, n_one=4):
    """The oracle as it stands, on bounded samples of the benchmark workload:
      - O_zoom (the method) on all host cores: store the blocks that the first
        nq queries touch, then answer those queries;
      - O_direct (Problem 1's ground truth, the SVD of the raw range rows) on
        all host cores for the first n_direct queries;
      - O_zoom on one thread: n_one queries on the same store, and the store
        of the blocks those queries touch."""
    import numpy as np

    import oracle

    oracle.load()
    cores = oracle.max_threads()
    # Sample: the first nq queries, re-based onto the span of rows they cover.
    ts = np.asarray(ts[:nq], np.int64)
    te = np.asarray(te[:nq], np.int64)
    lo_blk = int(ts.min()) // b
    hi_blk = (int(te.max()) - 1) // b + 1
    Asub = np.ascontiguousarray(A[lo_blk * b:min(hi_blk * b, A.shape[0])])
    a = time.perf_counter()
    st = oracle.store(Asub, b, k)
    store_s = time.perf_counter() - a
    a = time.perf_counter()
    oracle.query_batch(st, ts - lo_blk * b, te - lo_blk * b, k)
    query_s = time.perf_counter() - a
    log("cpu baseline: O_zoom %d queries in %.2f s (store %.2f s)" % (nq, query_s, store_s))
    # O_direct: the raw rows of each range, Householder QR then one-sided Jacobi.
    nd = min(n_direct, nq)
    a = time.perf_counter()
    oracle.direct_batch(Asub, ts[:nd] - lo_blk * b, te[:nd] - lo_blk * b, k)
    direct_s = time.perf_counter() - a
    log("cpu baseline: O_direct %d queries in %.2f s" % (nd, direct_s))
    # One thread.
    n1 = min(n_one, nq)
    oracle.set_threads(1)
    try:
        a = time.perf_counter()
        oracle.query_batch(st, ts[:n1] - lo_blk * b, te[:n1] - lo_blk * b, k)
        q1_s = time.perf_counter() - a
        b0 = int(ts[:n1].min()) // b
        b1 = (int(te[:n1].max()) - 1) // b + 1
        nb1 = min(b1 - b0, 64)
        A1 = np.ascontiguousarray(A[b0 * b:min((b0 + nb1) * b, A.shape[0])])
        a = time.perf_counter()
        oracle.store(A1, b, k)
        s1_s = time.perf_counter() - a
    finally:
        oracle.set_threads(cores)
    log("cpu baseline: one thread, %d queries in %.2f s, %d blocks in %.2f s" % (n1, q1_s, nb1, s1_s))
    qlen = int(te[0] - ts[0])
    return {"value": nq / query_s, "unit": "SVDs/s", "cores": cores, "kind": "oracle",
            "sample": "%d queries of %d rows over %d stored blocks (%d x %d f64); store %.2f s "
                      "(%.3f GB/s), queries %.2f s" % (nq, qlen, st.nb, Asub.shape[0],
                                                        Asub.shape[1], store_s,
                                                        Asub.nbytes / store_s / 1e9, query_s),
            "store_gbps": Asub.nbytes / store_s / 1e9,
            "direct": {"value": nd / direct_s, "unit": "SVDs/s", "cores": cores,
                       "kind": "oracle_direct",
                       "sample": "%d queries of %d rows: the SVD of the raw rows (Householder QR "
                                 "+ one-sided Jacobi)" % (nd, qlen), "seconds": direct_s},
            "one_thread": {"value": n1 / q1_s, "unit": "SVDs/s", "cores": 1, "kind": "oracle",
                           "sample": "%d queries of %d rows on the stored blocks; store of %d "
                                     "blocks" % (n1, qlen, nb1),
                           "store_gbps": A1.nbytes / s1_s / 1e9}}


if __name__ == "__main__":
    main()
