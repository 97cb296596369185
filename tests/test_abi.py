"""The C-ABI library loads and exports every function include/*.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1510_07522_amd", "librsrr.so")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(rsrr_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["rsrr_create", "rsrr_create_bem", "rsrr_sample", "rsrr_orthonormalize",
                     "rsrr_project", "rsrr_solve", "rsrr_result_info", "rsrr_result_copy",
                     "rsrr_result_free", "rsrr_destroy", "rsrr_last_error",
                     "rsrr_default_params", "rsrr_moment_matrix"]:
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="librsrr.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="librsrr.so not built")
def test_binding_signatures_cover_the_header():
    from paper_1510_07522_amd import _binding
    assert set(declared_functions()) == set(_binding.SIGNATURES)
    _binding.load()


@pytest.mark.skipif(not os.path.exists(LIB), reason="librsrr.so not built")
def test_default_params_and_error_paths_without_gpu():
    import paper_1510_07522_amd as P
    p = P.default_params()
    assert (p.NS, p.K, p.delta, p.tol_gap, p.tol_res) == (512, 2, 1e-14, 1e3, 1e-10)
    lib = P.load()
    # argument validation happens before any device call
    h = ctypes.c_void_p()
    st = lib.rsrr_create(ctypes.byref(h), 0, 1, None, None, None, None)
    assert st == -1
    assert b"null" in lib.rsrr_last_error() or b"n=" in lib.rsrr_last_error()


@pytest.mark.skipif(not os.path.exists(LIB), reason="librsrr.so not built")
def test_order_limits_are_checked_before_any_device_call():
    # complex64 factorisations go up to order 16384, complex128 ones to 8192
    import paper_1510_07522_amd as P
    from paper_1510_07522_amd import _binding
    lib = P.load()
    h = ctypes.c_void_p()
    kinds = (ctypes.c_int * 1)(0)
    ptrs = (ctypes.c_void_p * 1)(ctypes.c_void_p(1))
    fns = (_binding.fn_t * 1)()
    st = lib.rsrr_create(ctypes.byref(h), 16385, 1, kinds, ptrs, fns, None)
    assert st == -1 and b"16384" in lib.rsrr_last_error()
    xyz = (ctypes.c_double * 3)()
    st = lib.rsrr_create_bem(ctypes.byref(h), 16385, xyz, ctypes.c_double(0.1), None)
    assert st == -1 and b"16384" in lib.rsrr_last_error()
    one = ctypes.c_void_p(1)
    # precision 0 = complex128: 8193 is refused, before any allocation
    st = lib.rsrr_gesv_batched(0, 8193, 1, one, 8193, 0, one, 8193, 0, 1, 64, None, None)
    assert st == -1 and b"gesv" in lib.rsrr_last_error()
    st = lib.rsrr_gesv_batched(1, 16385, 1, one, 16385, 0, one, 16385, 0, 1, 64, None, None)
    assert st == -1 and b"gesv" in lib.rsrr_last_error()


@pytest.mark.skipif(not os.path.exists(LIB), reason="librsrr.so not built")
def test_load_shares_torchs_hip_runtime():
    # loading the library before torch is imported must not leave a second HIP
    # runtime in the process (torch's memory and streams would be foreign to it)
    import subprocess
    import sys
    code = ("import paper_1510_07522_amd as P; P.load(); import torch; "
            "m = open('/proc/self/maps').read(); "
            "print(len({l.split()[-1] for l in m.splitlines() if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"
