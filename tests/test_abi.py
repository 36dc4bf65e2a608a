"""The C-ABI library loads and exports every function include/sznb.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sznb.h")
LIB = os.path.join(ROOT, "paper_1711_03888_amd", "csrc", "libsznb.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sznb_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for need in ("sznb_compress", "sznb_decompress", "sznb_compress_batch", "sznb_decompress_batch",
                 "sznb_compress_bound", "sznb_read_status", "sznb_strerror", "sznb_stream_info"):
        assert need in names


def test_library_exports_all_declared_symbols():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_host_only_functions():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    from paper_1711_03888_amd import sznb
    L = sznb.lib()
    assert sznb.strerror(sznb.ECORRUPT) == "corrupt stream"
    n = 1 << 20
    assert L.sznb_compress_bound(n, sznb.PRED_LV) > 4 * n
    import oracle
    import numpy as np
    s = oracle.compress(np.arange(5000, dtype=np.float32), 1e-3, oracle.BESTFIT | oracle.EB_REL)
    info = sznb.stream_info(s[:128])
    assert info["n"] == 5000 and info["total_bytes"] == len(s)
    assert info["mode"] & 3 == oracle.BESTFIT and info["mode"] & sznb.EB_REL
