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
    # torch's HIP runtime first, so that a GPU test later in this process finds only that one
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    lib.dsve_abi_version.restype = ctypes.c_int
    assert lib.dsve_abi_version() == 5


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
    p.law = 7
    assert dsve.lib.dsve_init(ctypes.byref(h), ctypes.byref(p), 10, None) == dsve.E_ARG
    bad = [
        dict(law=dsve.LAW_MPM, A_g=0.0, law_extra=(3e-4, 2.6)),                 # no K_s
        dict(law=dsve.LAW_MPM, A_g=0.01, law_extra=(3e-4, 2.6), ks=40.0),       # A_g unused
        dict(law=dsve.LAW_MPM, A_g=0.0, law_extra=(3e-4, 1.0), ks=40.0),        # S_g <= 1
        dict(law=dsve.LAW_VANRIJN, A_g=0.0, law_extra=(3e-4, 2.6, 1e-6), ks=40.0),  # theta_cr
        dict(law=dsve.LAW_POWER, law_extra=(0.5,)),                             # beta < 1
        dict(law=dsve.LAW_GRASS_THR, law_extra=(-0.1,)),                        # u_cr < 0
        dict(law=dsve.LAW_GRASS, law_extra=(1.0,)),                             # unused entry
        dict(bc_right=dsve.BC_FIXED_DEPTH),                                      # no h_out
        dict(bc_left=dsve.BC_INFLOW_QH, q_in=0.1),                               # no h_in
        dict(bc_left=dsve.BC_DIRICHLET, bc_right=dsve.BC_DIRICHLET),            # no ghost depth
        dict(bc_left=6),
        dict(ks=-1.0),
    ]
    for kw in bad:
        p = dsve.make_params(dx=0.1, **kw)
        assert dsve.lib.dsve_init(ctypes.byref(h), ctypes.byref(p), 10, None) == dsve.E_ARG, kw
    p = dsve.make_params(dx=0.1, precision="mixed", solver="dot")
    assert dsve.lib.dsve_init(ctypes.byref(h), ctypes.byref(p), 10, None) == dsve.E_UNSUPPORTED
    p = dsve.make_params(dx=0.1, solver=2)
    assert dsve.lib.dsve_init(ctypes.byref(h), ctypes.byref(p), 10, None) == dsve.E_ARG
    chans = dsve.make_channels([0.01, 0.01], [0.4, 0.4], [0.1, 0.1], [0, 3], [0, 0])
    off = (ctypes.c_int64 * 3)(0, 5, 10)
    p = dsve.make_params()
    assert dsve.lib.dsve_batch_init(ctypes.byref(h), 2, off, chans, ctypes.byref(p), None) == dsve.E_ARG
    assert dsve.lib.dsve_destroy(None) == dsve.E_ARG
    assert dsve.lib.dsve_sync(None) == dsve.E_ARG


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdsve.so not built")
def test_struct_mirrors_match_the_header(tmp_path):
    # sizes and field offsets of the binding's ctypes structures against the C compiler's
    from paper_1912_04791_amd import dsve
    fields = {"dsve_params": dsve.Params, "dsve_channel": dsve.Channel}
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "dsve.h"', "int main(void) {"]
    for cname, py in fields.items():
        src.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            src.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    src.append("return 0; }")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)])
    out = dict(line.split() for line in subprocess.check_output([str(exe)], text=True).splitlines())
    for cname, py in fields.items():
        assert int(out[cname]) == ctypes.sizeof(py)
        for f, _ in py._fields_:
            assert int(out[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libdsve.so not built")
def test_binding_shares_torchs_hip_runtime_whatever_the_import_order():
    # imported before torch, the binding must still leave one HIP runtime in the process:
    # a second one would not know torch's streams and memory
    import subprocess
    import sys
    code = ("import paper_1912_04791_amd.dsve, torch\n"
            "print(len({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"
