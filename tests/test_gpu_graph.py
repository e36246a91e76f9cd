"""The batched query form and the storage phase captured into HIP graphs
(zs_query_batch_graph, zs_store_graph_create): every replay equals the eager
result bitwise, with the program's own eager work and synchronisations
between replays."""
import numpy as np
import pytest
import torch

from paper_1805_00754_amd import synth
from paper_1805_00754_amd import zoomsvd as zs
from tests.gpu_common import download_store, say, to_dev

pytestmark = pytest.mark.gpu


def _outputs(b):
    torch.cuda.synchronize()
    return [x.cpu().numpy().copy() for x in (b.U, b.S, b.V, b.k_out)]


@pytest.mark.parametrize("mode", ["fp64", "fp32"])
def test_graph_replays_equal_eager_batch(mode):
    zs.load()
    ser, cfg = synth.workload("sinmix_10k_x64_f64")
    if mode == "fp64":
        st = zs.zs_store_blocks(to_dev(ser.A), cfg["b"], cfg["k"])
    else:
        st = zs.zs_store_blocks(to_dev(ser.A, torch.float32), cfg["b"], cfg["k"],
                                mode=zs.ZS_MODE_FP32)
    rng = synth.rng_for(91)
    nq = 24
    L = rng.integers(1, 8000, size=nq)
    ts = np.array([rng.integers(0, st.t - l + 1) for l in L], np.int64)
    te = ts + L
    kq = rng.choice(np.array([3, 7, cfg["k"]], np.int32), size=nq)
    say("graph", mode, nq)
    ref = _outputs(zs.zs_query_batch(st, ts, te, kq))
    g = zs.zs_query_batch_graph(st, ts, te, kq)
    got = _outputs(g.out)                       # the eager pass inside graph creation
    for a, b in zip(got, ref):
        np.testing.assert_array_equal(a, b)
    other = None
    for rep in range(3):
        # the program's own work between replays: clear the outputs, run an
        # unrelated query, synchronise
        for x in (g.out.U, g.out.S, g.out.V):
            x.zero_()
        g.out.k_out.fill_(-1)
        other = zs.zs_query(st, 0, min(st.t, 3000 + 100 * rep), cfg["k"])
        torch.cuda.synchronize()
        g.launch()
        got = _outputs(g.out)
        for a, b in zip(got, ref):
            np.testing.assert_array_equal(a, b)
    assert other is not None
    g.free()
    st.free()


def test_graph_rejects_bad_range():
    zs.load()
    ser, cfg = synth.workload("sinmix_10k_x64_f64")
    st = zs.zs_store_blocks(to_dev(ser.A), cfg["b"], cfg["k"])
    with pytest.raises(zs.ZSError):
        zs.zs_query_batch_graph(st, [0, 5], [10, st.t + 1], 3)
    st.free()


@pytest.mark.parametrize("name,mode,tdtype", [("fp64", zs.ZS_MODE_FP64, torch.float64),
                                              ("bf16", zs.ZS_MODE_BF16, torch.bfloat16)])
def test_store_graph_replays_equal_eager_store(name, mode, tdtype):
    """The storage phase captured once: each replay recompresses the input's
    current contents, bitwise as zs_store_blocks on the same contents.  The
    input is rewritten in place between replays (three different series of
    one shape, a short last block, c > 128 so the wide eigen-solver and the
    Gram-tree leaves of that path are in the graph too)."""
    zs.load()
    t, c, b, k = 5_300, 160, 1_000, 12
    series = [synth.sinusoid_mixture(t, c, sources=10, seed=60 + i, noise="iid",
                                     noise_sigma=0.1, dtype="bf16" if name == "bf16" else "f64").A
              for i in range(3)]
    A = to_dev(series[0], tdtype)
    g = zs.zs_store_graph_create(A, b, k, mode=mode)
    torch.cuda.synchronize()
    say("store graph", name, (t, c, b, k))
    for rep in range(4):
        i = rep % 3
        ref_st = zs.zs_store_blocks(to_dev(series[i], tdtype), b, k, mode=mode)
        ref = download_store(ref_st)
        qref = [x.cpu() for x in zs.zs_query(ref_st, 123, 4_567, k)]
        ref_st.free()
        if rep > 0:
            A.copy_(to_dev(series[i], tdtype))     # the caller refreshes the input in place
            torch.cuda.synchronize()
            g.launch()
        zs.zs_sync_status(g.st)
        got = download_store(g.st)
        for x, y in zip(got, ref):
            np.testing.assert_array_equal(x, y)
        q = [x.cpu() for x in zs.zs_query(g.st, 123, 4_567, k)]
        for x, y in zip(q, qref):
            assert torch.equal(x, y)
    g.free()
    g.st.free()


def test_graph_replays_after_workspaces_released():
    """A captured batch owns its scratch: releasing the stream's workspaces
    (zs_release_workspaces) leaves its replays bitwise equal to the eager
    batch, and eager calls afterwards allocate again."""
    zs.load()
    ser, cfg = synth.workload("sinmix_10k_x64_f64")
    st = zs.zs_store_blocks(to_dev(ser.A), cfg["b"], cfg["k"])
    rng = synth.rng_for(93)
    ts, te = synth.queries_uniform(rng, st.t, 16, 50, 6_000)
    kq = np.full(16, cfg["k"], np.int32)
    ref = _outputs(zs.zs_query_batch(st, ts, te, kq))
    g = zs.zs_query_batch_graph(st, ts, te, kq)
    zs.zs_release_workspaces()
    say("replay after release")
    for x in (g.out.U, g.out.S, g.out.V):
        x.zero_()
    torch.cuda.synchronize()
    g.launch()
    for a, b in zip(_outputs(g.out), ref):
        np.testing.assert_array_equal(a, b)
    for a, b in zip(_outputs(zs.zs_query_batch(st, ts, te, kq)), ref):
        np.testing.assert_array_equal(a, b)
    g.free()
    st.free()
