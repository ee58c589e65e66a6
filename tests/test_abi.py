"""The C-ABI library loads on the host and exports every entry point of include/mfq.h."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mfq.h")
LIB = os.path.join(ROOT, "paper_2508_18468_amd", "libmfq.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mfq_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_api():
    names = declared_functions()
    for n in ("mfq_create", "mfq_init_state", "mfq_step", "mfq_entropy", "mfq_mutual_info"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmfq.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmfq.so not built")
def test_binding_covers_every_declared_symbol():
    from paper_2508_18468_amd import mfq
    assert sorted(mfq.EXPORTED) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libmfq.so not built")
def test_host_side_validation_without_gpu():
    """Calls that fail argument validation never touch the device."""
    from paper_2508_18468_amd import mfq
    l = mfq.lib()
    bad = mfq.Lattice(3, 8, 1, 0, 1.0)
    b = ctypes.c_size_t()
    assert l.mfq_workspace_bytes(ctypes.byref(bad), 4, 1, 0, ctypes.byref(b)) == -1
    ok = mfq.Lattice(1, 8, 1, 0, 1.0)
    assert l.mfq_workspace_bytes(ctypes.byref(ok), 8, 1, 0, ctypes.byref(b)) == -1  # N = L
    assert l.mfq_workspace_bytes(ctypes.byref(ok), 4, 0, 0, ctypes.byref(b)) == -1  # no trajectories
    assert l.mfq_workspace_bytes(ctypes.byref(ok), 4, 2, 0, ctypes.byref(b)) == 0
    assert b.value > 2 * 8 * 4 * 2 * 16
    assert l.mfq_destroy(None) == 0
    assert l.mfq_step(None, 0, None, 0.05, 0, 1) == -1
