"""The batched query form captured into a HIP graph (zs_query_batch_graph):
every replay equals the eager zs_query_batch result bitwise, with the
program's own eager work and synchronisations between replays."""
import numpy as np
import pytest
import torch

from paper_1805_00754_amd import synth
from paper_1805_00754_amd import zoomsvd as zs
from tests.gpu_common import say, to_dev

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
