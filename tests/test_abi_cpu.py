"""CPU-side checks of the boundary: the HIP library loads without a GPU and
exports every entry point include/clgc.h declares; argument validation that
happens before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "clgc.h")
LIB = os.path.join(ROOT, "paper_1311_1056_amd", "libclgc.so")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:cl_status|const char\*)\s+(cl_\w+)\s*\(", text, re.M)))


def test_header_declares_core_calls():
    syms = declared_symbols()
    for name in ("cl_lattice_create", "cl_langevin_step", "cl_gauge_cool", "cl_unitarity_norm",
                 "cl_measure", "cl_last_error"):
        assert name in syms


@pytest.mark.skipif(not os.path.exists(LIB), reason="libclgc.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libclgc.so not built")
def test_descriptor_validation_without_gpu():
    import paper_1311_1056_amd as cl
    n = cl.cl_lattice_bytes(cl.make_desc((4, 4, 4, 4), 6.0))
    n32 = cl.cl_lattice_bytes(cl.make_desc((4, 4, 4, 4), 6.0, precision=cl.CL_MIXED))
    assert n32 < n
    # links + drift + clover: (72 + 72 + 108) reals per site
    assert n >= 256 * 252 * 8
    for dims in ((3, 4, 4, 4), (4, 4, 4, 0), (4, 4, 5, 4)):
        with pytest.raises(cl.ClError) as e:
            cl.cl_lattice_bytes(cl.make_desc(dims, 6.0))
        assert e.value.status == cl.CL_EINVAL
    with pytest.raises(cl.ClError):
        cl.cl_lattice_bytes(cl.make_desc((4, 4, 4, 4), -1.0))
    with pytest.raises(cl.ClError):
        cl.cl_lattice_bytes(cl.make_desc((4, 4, 4, 4), 6.0, precision=7))
