"""Host-side checks of the C ABI (no GPU needed): the library loads and
exports every function that include/omg.h and include/omg_inspect.h declare,
and the binding's ctypes structures have the C layout of the header's
structures."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "omg.h")
HEADERS = [HEADER, os.path.join(ROOT, "include", "omg_inspect.h")]
LIB = os.path.join(ROOT, "paper_2512_08728_amd", "libomg.so")


def declared(headers=HEADERS):
    names = set()
    for h in headers:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(omg_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_boundary():
    """omg.h holds the solve boundary (setup from a matrix and a hierarchy,
    setup from a coefficient field, solve, batched solve, backward, destroy)
    and its helpers; the inspection hooks live in omg_inspect.h."""
    names = declared([HEADER])
    for n in ("omg_setup", "omg_setup_sip", "omg_solve", "omg_solve_batched", "omg_solve_backward",
              "omg_destroy", "omg_strerror", "omg_grid_hierarchy", "omg_embedding"):
        assert n in names
    assert not any(n.startswith(("omg_level_", "omg_probe", "omg_bench", "omg_get_")) for n in names)


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


def test_struct_layout_matches_header(tmp_path):
    """Compile a C program against include/omg.h (gcc) that prints the size
    and every field offset of the option, report, grid and BSR structures;
    the ctypes mirrors must agree field by field."""
    import paper_2512_08728_amd as omg
    mirrors = {"omg_options": omg.Options, "omg_report": omg.Report, "omg_grid": omg.Grid, "omg_bsr": omg.Bsr,
               "omg_hierarchy": omg.HierarchyC}
    lines = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void) {"]
    for cname, cls in mirrors.items():
        lines.append(f'    printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'    printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("    return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-o", str(exe), str(src)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, cls in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


def test_option_names_map_to_header_values():
    import paper_2512_08728_amd as omg
    if not os.path.exists(LIB):
        pytest.skip("libomg.so not built")
    o = omg.options(variant="hybrid", smoother="schwarz", n_s_max=5, precision="mixed_flex")
    assert (o.variant, o.smoother, o.n_s_max, o.precision) == (omg.HYBRID, omg.SMOOTH_AS, 5, omg.MIXED_FLEX)
    src = open(HEADER).read()
    for name, val in (("OMG_SYNC_MULT", omg.SYNC_MULT), ("OMG_OVERLAP_DET", omg.OVERLAP_DET),
                      ("OMG_HYBRID", omg.HYBRID), ("OMG_ADD_SYNC", omg.ADD_SYNC), ("OMG_SMOOTH_BJ", omg.SMOOTH_BJ),
                      ("OMG_SMOOTH_AS", omg.SMOOTH_AS), ("OMG_MIXED_FLEX", omg.MIXED_FLEX)):
        assert re.search(rf"\b{name}\s*=\s*{val}\b", src), name
