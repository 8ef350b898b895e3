"""Host-side checks of the C ABI (no GPU needed): the library loads and
exports every function that include/omg.h declares."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "omg.h")
LIB = os.path.join(ROOT, "paper_2512_08728_amd", "libomg.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(omg_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("omg_setup", "omg_setup_sip", "omg_solve", "omg_solve_batched", "omg_solve_backward",
              "omg_destroy", "omg_strerror"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("libomg.so not built")
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (omg_[a-z_0-9]+)$", out, flags=re.M))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing
    lib = ctypes.CDLL(LIB)  # loads without a GPU
    for n in declared():
        assert hasattr(lib, n)


def test_binding_names_match_header():
    import paper_2512_08728_amd as omg
    assert sorted(omg.EXPORTS) == declared()


def test_strerror_and_defaults_without_gpu():
    if not os.path.exists(LIB):
        pytest.skip("libomg.so not built")
    import paper_2512_08728_amd as omg
    o = omg.options()
    assert o.omega == 0.7 and o.crit_rel[0] == 0.1 and o.crit_max[0] == 20
    assert o.crit_rel[1] == 0.5 and o.crit_max[1] == 2 and o.crit_max[2] == 1
    assert omg.lib().omg_strerror(omg.ENOTSPD) == b"matrix not symmetric positive definite"
