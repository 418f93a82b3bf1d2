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


@pytest.mark.skipif(not os.path.exists(LIB), reason="libclgc.so not built")
def test_maximum_sizes_without_gpu():
    """Every field must stay below 4 GiB (one 32-bit buffer resource): the
    clover field, 864 V bytes in FP64 and 432 V in mixed precision, sets the
    largest lattice, 46^4 (FP64) and 56^4 (mixed); the next even sizes are
    refused.  Chains: 1..1024 links, 1..2^24 chains."""
    import paper_1311_1056_amd as cl
    assert cl.cl_lattice_bytes(cl.make_desc((46, 46, 46, 46), 6.0)) > 9 * 10**9
    assert cl.cl_lattice_bytes(cl.make_desc((56, 56, 56, 56), 6.0, precision=cl.CL_MIXED)) > 9 * 10**9
    for dims, prec in (((48, 48, 48, 48), cl.CL_FP64), ((58, 58, 58, 58), cl.CL_MIXED),
                       ((46, 46, 46, 52), cl.CL_FP64)):
        with pytest.raises(cl.ClError) as e:
            cl.cl_lattice_bytes(cl.make_desc(dims, 6.0, precision=prec))
        assert e.value.status == cl.CL_EINVAL
    lib = cl.lib
    for n, nc, ok in ((1024, 1, True), (1025, 1, False), (0, 1, False), (16, 1 << 24, True), (16, (1 << 24) + 1, False),
                      (16, 0, False)):
        d = cl.cl_chain_desc()
        d.n_links, d.n_chains, d.beta_re, d.beta_im = n, nc, 2.0, 1.0
        nbytes = ctypes.c_size_t(0)
        st = lib.cl_chain_bytes(ctypes.byref(d), ctypes.byref(nbytes))
        assert (st == 0) == ok, (n, nc, st)

