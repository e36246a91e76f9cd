"""CPU checks of the boundary: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "zoomsvd.h")


@pytest.fixture(scope="module")
def zs():
    from paper_1805_00754_amd import zoomsvd
    if not os.path.exists(zoomsvd.LIB_PATH):
        from paper_1805_00754_amd import build
        build.build()
    zoomsvd.load()
    return zoomsvd


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(zs_[a-z_]+)\s*\(", src)))


def test_header_declarations_are_exported(zs):
    names = declared_functions()
    assert "zs_store_blocks" in names and "zs_query" in names and "zs_query_batch" in names
    lib = ctypes.CDLL(zs.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), "missing export " + n
    assert sorted(zs.EXPORTED) == names


def test_version_and_error_string(zs):
    assert zs.zs_version().startswith("zoomsvd")
    assert isinstance(zs.zs_last_error(), str)


def test_store_rejects_bad_arguments(zs):
    lib = zs.load()
    vp = ctypes.c_void_p
    out = vp()
    A = vp(0x1000)   # never dereferenced: validation happens first
    cases = [
        (vp(0), 10, 4, 4, 0, 2, 2, 0, zs.ZS_EINVAL),     # null A
        (A, 0, 4, 4, 0, 2, 2, 0, zs.ZS_EINVAL),          # t < 1
        (A, 10, 4, 3, 0, 2, 2, 0, zs.ZS_EINVAL),         # lda < c
        (A, 10, 4, 4, 0, 0, 2, 0, zs.ZS_EINVAL),         # b < 1
        (A, 10, 4, 4, 0, 2, 0, 0, zs.ZS_EINVAL),         # k < 1
        (A, 10, 4, 4, 0, 2, 5, 0, zs.ZS_EINVAL),         # k > c
        (A, 10, 4096, 4096, 0, 2, 2, 0, zs.ZS_EUNSUPPORTED),  # c above the build limit
    ]
    for args in cases:
        st = lib.zs_store_blocks(*args[:8], vp(0), ctypes.byref(out))
        assert st == args[8], (args, st, zs.zs_last_error())
        assert out.value is None
        assert zs.zs_last_error()
    assert lib.zs_store_blocks(A, 10, 4, 4, 0, 2, 2, 0, vp(0), None) == zs.ZS_EINVAL


def test_store_xi_rejects_bad_threshold(zs):
    lib = zs.load()
    vp = ctypes.c_void_p
    out = vp()
    A = vp(0x1000)   # never dereferenced: validation happens first
    for xi in (-0.1, 1.5, float("nan")):
        assert lib.zs_store_blocks_xi(A, 10, 4, 4, 0, 2, 2, 0, xi, vp(0), ctypes.byref(out)) \
            == zs.ZS_EINVAL, xi
        assert out.value is None
    assert "xi" in zs.zs_last_error()


def test_window_similarity_rejects_bad_arguments(zs):
    lib = zs.load()
    vp = ctypes.c_void_p
    assert lib.zs_window_similarity(vp(0), 10, 20, 5, 2, vp(8), vp(0)) == zs.ZS_EINVAL
    assert lib.zs_window_similarity(vp(8), 10, 20, 5, 2, vp(0), vp(0)) == zs.ZS_EINVAL


def test_query_rejects_null_store(zs):
    lib = zs.load()
    vp = ctypes.c_void_p
    assert lib.zs_query(vp(0), 0, 1, 1, vp(8), 1, vp(8), vp(8), 1, vp(8), vp(0)) == zs.ZS_EINVAL
    assert lib.zs_query_noalloc(vp(0), 0, 1, 1, vp(8), 1, vp(8), vp(8), 1, vp(8), vp(0)) \
        == zs.ZS_EINVAL
    assert lib.zs_query_batch(vp(0), 1, vp(8), vp(8), vp(8), vp(8), vp(8), vp(8), vp(8), vp(8),
                              vp(8), vp(8), vp(0)) == zs.ZS_EINVAL
    assert lib.zs_store_bytes(vp(0)) == 0
    lib.zs_store_free(vp(0))   # no-op


def test_product_does_not_import_oracle():
    """The product package never touches the oracle (test infrastructure)."""
    pkg = os.path.join(ROOT, "paper_1805_00754_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", txt, re.M), f
                assert "liboracle" not in txt and "zoom_oracle" not in txt, f
