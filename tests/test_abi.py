"""The C ABI library loads, exports every declared symbol and rejects bad
arguments before touching the GPU (runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    import paper_2506_03266_amd.binding as b
    if not os.path.exists(b.LIB_PATH):
        from paper_2506_03266_amd import build
        build.build()
    return b.lib()


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(mpd_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_exports_every_declared_symbol(lib):
    names = declared_symbols()
    assert "mpd_decode_batch" in names and len(names) >= 6
    for name in names:
        assert hasattr(lib, name), name


def test_version_and_workspace(lib):
    assert lib.mpd_version().startswith(b"mpd")
    assert lib.mpd_workspace_bytes(64, 10000) == 0           # on-chip path
    assert lib.mpd_workspace_bytes(256, 0) == 0
    w1 = lib.mpd_workspace_bytes(256, 1)
    w2 = lib.mpd_workspace_bytes(256, 4096)
    assert w1 > 2 * 256 * 256 * 8 and w2 > 4096 * 2 * 256 * 256 * 8


@pytest.mark.parametrize("L,p,n,T,code", [
    (2, 0.1, 1, 8, -1), (1025, 0.1, 1, 8, -1), (200, 0.1, 1, 8, -1), (127, 0.1, 1, 8, -1),
    (16400, 0.1, 1, 8, -1),
    (16, -0.1, 1, 8, -2), (16, 1.5, 1, 8, -2), (16, float("nan"), 1, 8, -2),
    (16, 0.1, 1, -1, -3), (16, 0.1, 1, 10923, -3),
    (16, 0.1, -1, 8, -7),
])
def test_bad_arguments_rejected(lib, L, p, n, T, code):
    dummy = ctypes.c_void_p(4096)  # never dereferenced: validation fails first
    rc = lib.mpd_decode_batch(L, p, dummy, n, T, dummy, dummy, None, None, 0, None)
    assert rc == code
    assert len(lib.mpd_last_error()) > 0


def test_null_pointers_rejected(lib):
    rc = lib.mpd_decode_batch(16, 0.1, None, 4, 8, None, None, None, None, 0, None)
    assert rc == -4
    dummy = ctypes.c_void_p(4096)
    rc = lib.mpd_decode_batch(256, 0.1, dummy, 4, 8, dummy, dummy, None, None, 0, None)
    assert rc == -5  # workspace missing for the tiled path


def test_empty_batch_is_a_noop(lib):
    assert lib.mpd_decode_batch(16, 0.1, None, 0, 8, None, None, None, None, 0, None) == 0
