"""The C ABI library loads and exports every entry point its header declares
(no GPU needed: nothing is called except the pure host queries)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "aframe_mi.h")
LIB = os.path.join(ROOT, "paper_2403_18661_amd", "libaframe_mi.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(af_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def so():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} not built (python -m paper_2403_18661_amd.build)")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(so):
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(so, n), n


def test_binding_covers_the_header():
    from paper_2403_18661_amd._lib import SIGNATURES
    assert set(declared_functions()) == set(SIGNATURES)


def test_host_queries(so):
    so.af_version.restype = ctypes.c_char_p
    assert b"gfx950" in so.af_version()
    so.af_psd_workspace_bytes.restype = ctypes.c_size_t
    so.af_psd_workspace_bytes.argtypes = [ctypes.c_int64] * 6
    # 15 segments x 2 channels x 2049 bins x 8 bytes
    assert so.af_psd_workspace_bytes(2, 4096, 2048, 32768, 0, 1) >= 15 * 2 * 2049 * 8
    assert so.af_psd_workspace_bytes(2, 3000, 1500, 32768, 0, 1) == 0      # not a power of two
    so.af_whiten_workspace_bytes.restype = ctypes.c_size_t
    so.af_whiten_workspace_bytes.argtypes = [ctypes.c_int64] * 3
    assert so.af_whiten_workspace_bytes(2, 4096, 451) >= 451 * 2 * 4097 * 4
