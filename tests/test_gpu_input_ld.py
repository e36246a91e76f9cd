"""A store built from rows with a leading dimension larger than c (a column
slice of a wider array) equals, bit for bit, the store of the same values laid
out densely: the storage phase reads each row at its own start, in the same
order, whatever the row pitch.  Odd pitches leave FP64 rows only 8-byte
aligned and FP32 rows 4-byte aligned, so the 16-byte row reads of the
projection run on unaligned rows; c = 64 takes the whole-panel path and
c = 40 the clamped one (c not a multiple of 16)."""
import numpy as np
import pytest
import torch

from paper_1805_00754_amd import synth
from paper_1805_00754_amd import zoomsvd as zs
from tests.gpu_common import download_store, say

pytestmark = pytest.mark.gpu

CASES = [("f64", torch.float64, zs.ZS_MODE_FP64), ("f32", torch.float32, zs.ZS_MODE_FP32),
         ("bf16", torch.bfloat16, zs.ZS_MODE_BF16)]


@pytest.mark.parametrize("name,tdtype,mode", CASES)
@pytest.mark.parametrize("c,pad", [(64, 3), (40, 1)])
def test_padded_rows_equal_dense(name, tdtype, mode, c, pad):
    zs.load()
    t, b, k = 3_000, 300, 12
    ser = synth.sinusoid_mixture(t, c, sources=6, seed=21 + c, noise="iid", noise_sigma=0.1,
                                 dtype=name)
    dense = torch.from_numpy(ser.A).cuda().to(tdtype).contiguous()
    wide = torch.zeros((t, c + pad), dtype=tdtype, device="cuda")
    wide[:, :c] = dense
    view = wide[:, :c]
    assert view.stride(0) == c + pad
    say("input ld", name, c, pad)
    st_d = zs.zs_store_blocks(dense, b, k, mode=mode)
    st_w = zs.zs_store_blocks(view, b, k, mode=mode)
    torch.cuda.synchronize()
    for x, y in zip(download_store(st_d), download_store(st_w)):
        np.testing.assert_array_equal(x, y)
    ts, te = 137, 2_611
    a = [x.cpu() for x in zs.zs_query(st_d, ts, te, k)]
    w = [x.cpu() for x in zs.zs_query(st_w, ts, te, k)]
    for x, y in zip(a, w):
        assert torch.equal(x, y)
    st_d.free()
    st_w.free()
