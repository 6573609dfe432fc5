"""The C-ABI library loads on the CPU and exports every symbol include/dsve.h declares.

No compute calls are made (no GPU here); the GPU tests call through the same ABI.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dsve.h")
LIB = os.path.join(ROOT, "paper_1912_04791_amd", "libdsve.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([a-z_][a-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("dsve_init", "dot_edge_fluct", "cell_update", "cfl_reduce", "adot_step",
                 "dsve_batch_init", "adot_step_batched", "dsve_sync", "dsve_last_error",
                 "dsve_destroy", "dsve_autotune", "dsve_set_launch"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdsve.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    lib.dsve_abi_version.restype = ctypes.c_int
    assert lib.dsve_abi_version() == 1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdsve.so not built")
def test_binding_lists_all_entry_points():
    from paper_1912_04791_amd import dsve
    assert set(declared_functions()) == set(dsve.ENTRY_POINTS)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdsve.so not built")
def test_argument_errors_without_device_work():
    # argument validation happens before any HIP call
    from paper_1912_04791_amd import dsve
    h = ctypes.c_void_p()
    p = dsve.make_params(dx=0.1)
    assert dsve.lib.dsve_init(ctypes.byref(h), ctypes.byref(p), 0, None) == dsve.E_ARG
    p = dsve.make_params(dx=0.1, n_gauss=7)
    assert dsve.lib.dsve_init(ctypes.byref(h), ctypes.byref(p), 10, None) == dsve.E_ARG
    p = dsve.make_params(dx=0.1, porosity=1.0)
    assert dsve.lib.dsve_init(ctypes.byref(h), ctypes.byref(p), 10, None) == dsve.E_ARG
    p = dsve.make_params(dx=0.1, bc_left=dsve.BC_PERIODIC)
    assert dsve.lib.dsve_init(ctypes.byref(h), ctypes.byref(p), 10, None) == dsve.E_ARG
    p = dsve.make_params(dx=0.1)
    p.law = 3
    assert dsve.lib.dsve_init(ctypes.byref(h), ctypes.byref(p), 10, None) == dsve.E_UNSUPPORTED
    assert dsve.lib.dsve_destroy(None) == dsve.E_ARG
    assert dsve.lib.dsve_sync(None) == dsve.E_ARG
