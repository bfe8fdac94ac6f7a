"""The C-ABI library: it is built, loads, and exports every symbol the header declares.

CPU only: nothing here launches GPU work.
"""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lqcd.h")
LIB = os.path.join(ROOT, "paper_2303_05883_amd", "liblqcd.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lqcd_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["lqcd_create", "lqcd_destroy", "lqcd_set_gauge", "lqcd_set_clover", "lqcd_apply",
                     "lqcd_solve", "lqcd_solve_batch", "lqcd_apply_native", "lqcd_import", "lqcd_export"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("liblqcd.so not built: run python -m paper_2303_05883_amd.build")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_the_same_symbols():
    from paper_2303_05883_amd import lqcd
    assert sorted(lqcd.EXPORTED) == declared_functions()


def test_host_only_entry_points():
    from paper_2303_05883_amd import lqcd
    lib = lqcd.load()
    assert lib.lqcd_strerror(0) == b"ok"
    assert lib.lqcd_strerror(-7) == b"gauge link is not SU(3)"
    p = lqcd.default_params()
    assert p.tol == 1e-10 and p.inner_prec == lqcd.F64 and p.check_every == 8 and p.use_graph == 1
    # argument errors are caught before any device call
    h = ctypes.c_void_p()
    bad = (ctypes.c_int * 4)(4, 4, 3, 4)
    assert lib.lqcd_create(bad, -1, None, ctypes.byref(h)) == lqcd.EINVAL
    assert b"even" in lib.lqcd_last_error()
    good = (ctypes.c_int * 4)(4, 4, 4, 4)
    assert lib.lqcd_create(good, 0, None, ctypes.byref(h)) == lqcd.EINVAL
    assert lib.lqcd_set_clover(None, 0.1, 0.0) == lqcd.EINVAL
    assert lib.lqcd_apply(None, 0, 0, None, None, 0) == lqcd.EINVAL
    # batched entry points: no lattices, too many lattices, null lists
    one = (ctypes.c_int * 1)(1)
    assert lib.lqcd_solve_batch(None, one, None, None, 0, None, None) == lqcd.EINVAL
    assert lib.lqcd_solve_batch(None, one, None, None, 17, None, None) == lqcd.EINVAL
    assert lib.lqcd_batch_autotune(None, one, 1, 3, None, None) == lqcd.EINVAL
    g = ctypes.c_double()
    assert lib.lqcd_bandwidth_probe(None, 0, 1 << 20, 1, ctypes.byref(g)) == lqcd.EINVAL


def test_single_hip_runtime_in_process():
    """Loading the library must not bring a second HIP runtime next to torch's
    (a torch stream passed to another runtime instance crashes the process)."""
    import subprocess
    import sys
    code = ("from paper_2303_05883_amd import lqcd; lqcd.load(); import torch; "
            "m = open('/proc/self/maps').read().splitlines(); "
            "print(len({l.split()[-1] for l in m if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "1"
