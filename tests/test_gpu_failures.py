"""Failure paths of the C ABI forced from the host: a Jacobi sweep cap of 1
makes the store call and zs_sync_status report ZS_ENOCONV (every kernel
still exits normally), and a store larger than the device memory is refused
with ZS_ENOMEM before anything is allocated or launched."""
import ctypes

import pytest
import torch

from paper_1805_00754_amd import synth
from paper_1805_00754_amd import zoomsvd as zs
from tests.gpu_common import say, to_dev

pytestmark = pytest.mark.gpu


def test_sweep_cap_forces_enoconv():
    zs.load()
    A = synth.sinusoid_mixture(3_000, 64, sources=8, seed=5, noise="iid", noise_sigma=0.1).A
    dA = to_dev(A)
    st = zs.zs_store_blocks(dA, 500, 10)
    try:
        zs.zs_set_sweep_cap(1)
        say("store with sweep cap 1")
        with pytest.raises(zs.ZSError) as ei:
            zs.zs_store_blocks(dA, 500, 10)
        assert ei.value.status == zs.ZS_ENOCONV
        say("query with sweep cap 1")
        zs.zs_query(st, 123, 2_877, 10)
        with pytest.raises(zs.ZSError) as ei:
            zs.zs_sync_status(st)
        assert ei.value.status == zs.ZS_ENOCONV
    finally:
        zs.zs_set_sweep_cap(40)
    # the flag was cleared when it was reported; the default cap converges
    zs.zs_query(st, 123, 2_877, 10)
    zs.zs_sync_status(st)
    zs.zs_store_blocks(dA, 500, 10).free()
    with pytest.raises(zs.ZSError) as ei:
        zs.zs_set_sweep_cap(0)
    assert ei.value.status == zs.ZS_EINVAL
    st.free()


def test_store_beyond_device_memory_is_enomem():
    lib = zs.load()
    A = torch.zeros((4, 64), dtype=torch.float64, device="cuda")
    out = ctypes.c_void_p()
    # 2^40 rows: 128 TB of U alone; refused on the host, A is never read
    s = lib.zs_store_blocks(ctypes.c_void_p(A.data_ptr()), 1 << 40, 64, 64, zs.ZS_F64, 1_000, 16,
                            zs.ZS_MODE_FP64, ctypes.c_void_p(0), ctypes.byref(out))
    assert s == zs.ZS_ENOMEM, zs.zs_last_error()
    assert out.value is None
    assert "device" in zs.zs_last_error()
    # the library is still usable
    small = synth.sinusoid_mixture(1_000, 16, sources=4, seed=1, noise="iid").A
    zs.zs_store_blocks(to_dev(small), 100, 4).free()
