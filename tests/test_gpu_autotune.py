"""The launch-variant autotuner: every variant of every tuned site computes
the same bits (forced one by one on the same store and batch), the tuner
records a choice per shape, and a choice written to the ZS_AUTOTUNE_CACHE
file is reused by the next process without timing again."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

from paper_1805_00754_amd import synth
from paper_1805_00754_amd import zoomsvd as zs
from tests.gpu_common import download_store, say, to_dev

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SITES = {"gram_lp_tile": 2, "eig_tri_threads": 2, "blockprod_order": 2, "stack_order": 2}


def _run(A, tdtype, b, k, mode, ts, te, kq):
    st = zs.zs_store_blocks(to_dev(A, tdtype), b, k, mode=mode)
    out = zs.zs_query_batch(st, ts, te, kq)
    torch.cuda.synchronize()
    res = list(download_store(st)) + [x.cpu().numpy().copy() for x in (out.U, out.S, out.V, out.k_out)]
    st.free()
    return res


@pytest.mark.parametrize("c,b,k,mode,tdtype", [(128, 500, 16, zs.ZS_MODE_FP32, torch.float32),
                                                (256, 1000, 20, zs.ZS_MODE_BF16, torch.bfloat16)])
def test_forced_variants_compute_the_same_bits(c, b, k, mode, tdtype):
    zs.load()
    t = 6 * b + 123
    A = synth.sinusoid_mixture(t, c, sources=12, seed=c, noise="iid", noise_sigma=0.1,
                               dtype="f32" if tdtype == torch.float32 else "bf16").A
    ts, te = synth.queries_uniform(synth.rng_for(c + 1), t, 300, 1, t)
    kq = np.full(len(ts), k, np.int32)
    try:
        for site in SITES:
            zs.zs_autotune_force(site, 0)
        ref = _run(A, tdtype, b, k, mode, ts, te, kq)
        for site, n in SITES.items():
            for v in range(1, n):
                say("autotune variants", c, site, v)
                zs.zs_autotune_force(site, v)
                got = _run(A, tdtype, b, k, mode, ts, te, kq)
                for x, y in zip(got, ref):
                    np.testing.assert_array_equal(x, y)
                zs.zs_autotune_force(site, 0)
    finally:
        for site in SITES:
            zs.zs_autotune_force(site, -1)


CHILD = r"""
import json, sys
sys.path.insert(0, %r)
import numpy as np, torch
from paper_1805_00754_amd import synth, zoomsvd as zs
zs.load()
A = synth.sinusoid_mixture(4_100, 256, sources=8, seed=3, noise="iid", noise_sigma=0.1, dtype="bf16").A
st = zs.zs_store_blocks(torch.from_numpy(A).cuda().to(torch.bfloat16), 1000, 16, mode=zs.ZS_MODE_BF16)
ts, te = synth.queries_uniform(synth.rng_for(4), 4_100, 40, 1, 4_100)
zs.zs_query_batch(st, ts, te, 16)
torch.cuda.synchronize()
print(json.dumps({k: list(v) for k, v in zs.zs_autotune_table().items()}))
"""


def test_cache_file_is_written_and_reused(tmp_path):
    cache = tmp_path / "tune.txt"
    env = dict(os.environ, ZS_AUTOTUNE_CACHE=str(cache), ZS_AUTOTUNE="1")
    code = CHILD % ROOT

    def child():
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                           timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        return json.loads(r.stdout.strip().splitlines()[-1])

    first = child()
    say("autotune table", first)
    sites = {k.split("|")[0] for k in first}
    assert {"gram_lp_tile", "blockprod_order"} <= sites
    lines = cache.read_text().splitlines()
    assert len(lines) == len(first)
    second = child()
    # the second process made no new choice: the file is unchanged and the
    # choices (and the timings they came with) are those of the first
    assert cache.read_text().splitlines() == lines
    assert second == first
