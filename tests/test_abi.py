"""The C-ABI library loads and exports every entry point include/pdsink.h declares.

CPU-only: loading libpdsink.so needs the HIP runtime library, not a GPU.
No compute entry point is called here.
"""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pdsink.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_operations():
    names = header_functions()
    for op in ("pd_discretize", "sinkhorn_dist_batch", "sinkhorn_dist_bounds_batch", "pd_barycenter",
               "kmeans_assign", "kmeans_lloyd"):
        assert op in names
    assert "pdsink_ctx_create" in names and "pdsink_strerror" in names


def test_library_exports_every_header_symbol():
    from paper_1805_08331_amd import _lib
    lib = _lib.load()
    for name in header_functions():
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, f"{name} has no ctypes signature"
    assert set(_lib.SIGNATURES) == set(header_functions())


def test_exported_dynamic_symbols_are_c_names():
    import subprocess
    from paper_1805_08331_amd import _lib
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    for name in header_functions():
        assert name in exported, name


def test_strerror_and_host_side_validation():
    """Argument errors are caught on the host before any device work."""
    import ctypes
    from paper_1805_08331_amd import _lib
    lib = _lib.load()
    assert lib.pdsink_strerror(0) == b"ok"
    assert lib.pdsink_strerror(-1) == b"invalid argument"
    out = ctypes.c_void_p()
    bad = [
        _lib.Params(1, 2.0, 1e-3, 1e-3, 100, 0, 1e-3),     # d < 2
        _lib.Params(257, 2.0, 1e-3, 1e-3, 100, 0, 1e-3),   # d > 256
        _lib.Params(32, 2.0, 5e-6, 1e-3, 100, 0, 1e-3),    # gamma below the scale range
        _lib.Params(32, 0.5, 1e-3, 1e-3, 100, 0, 1e-3),    # p < 1
        _lib.Params(32, 2.0, 0.0, 1e-3, 100, 0, 1e-3),     # gamma <= 0
        _lib.Params(32, 2.0, 1e-3, -1.0, 100, 0, 1e-3),    # tol < 0
        _lib.Params(32, 2.0, 1e-3, 1e-3, 0, 0, 1e-3),      # max_iter < 1
        _lib.Params(32, 2.0, 1e-3, 1e-3, 100, 7, 1e-3),    # unknown precision
        _lib.Params(64, 2.0, 1e-3, 1e-3, 100, 0, 1e-3, 7),   # unknown kernel
        _lib.Params(32, 2.0, 1e-3, 1e-3, 100, 0, 1e-3, 1),   # resident kernel below its grids
        _lib.Params(101, 2.0, 1e-3, 1e-3, 100, 0, 1e-3, 1),  # resident kernel above its grids
    ]
    for prm in bad:
        assert lib.pdsink_ctx_create(ctypes.byref(prm), 0, ctypes.byref(out)) == _lib.PDSINK_EINVAL
        assert not out.value
    assert lib.pdsink_ctx_create(None, 0, ctypes.byref(out)) == _lib.PDSINK_EINVAL
    # NULL context
    n = ctypes.c_size_t()
    assert lib.pdsink_workspace_bytes(None, 0, 10, ctypes.byref(n)) == _lib.PDSINK_EINVAL
    assert lib.sinkhorn_dist_batch(None, 1, None, None, None, None, None, None, None, None, None, None, 0,
                                   None) == _lib.PDSINK_EINVAL
    assert lib.sinkhorn_dist_batch_noalloc(None, 1, None, None, None, None, None, None, None, None,
                                           None) == _lib.PDSINK_EINVAL
    assert lib.sinkhorn_dist_batch_notify(None, 1, None, None, None, None, None, None, None, None, None, 1, None,
                                          0, None) == _lib.PDSINK_EINVAL
    assert lib.sinkhorn_dist_bounds_batch(None, 1, None, None, None, None, None, None, None, None, None, None,
                                          None, 0, None) == _lib.PDSINK_EINVAL
    assert lib.pd_discretize(None, None, None, 1, None, None, None, None) == _lib.PDSINK_EINVAL
    assert lib.kmeans_assign(None, 1, None, 1, None, None, None, None, None, 0, None) == _lib.PDSINK_EINVAL
    e, o = ctypes.c_double(), ctypes.c_int32()
    assert lib.pd_barycenter(None, 1, None, 5.0, 10, 0.01, 1, None, ctypes.byref(e), ctypes.byref(o), None, 0,
                             None) == _lib.PDSINK_EINVAL
    assert lib.pd_sharpen(None, 1, None, 1.0, None, None) == _lib.PDSINK_EINVAL
    assert lib.pd_quantize(None, 1, None, None, None) == _lib.PDSINK_EINVAL
    assert lib.kmeans_lloyd(None, 1, None, 1, None, 1, 5.0, 10, 0.01, None, None, None, None, 0,
                            None) == _lib.PDSINK_EINVAL
    assert lib.pdsink_strerror(_lib.PDSINK_ERANGE) != lib.pdsink_strerror(_lib.PDSINK_EINVAL)


def test_product_package_does_not_import_the_oracle():
    """The GPU path never routes through the oracle (or any CPU fallback)."""
    pkg = os.path.join(ROOT, "paper_1805_08331_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", src, flags=re.M), f
                assert "oracle." not in src or f.endswith((".hip", ".h")), f
