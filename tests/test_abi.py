"""The C-ABI library loads and exports every entry point declared in
include/msplit.h; host-side logic that needs no GPU (counts, status text)."""
import ctypes
import os
import re
import subprocess

import pytest

from oracle import counts

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "msplit.h")
LIB = os.path.join(ROOT, "paper_2402_06083_amd", "libmsplit.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(msplit_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2402_06083_amd import _build
        _build.build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 8
    for name in names:
        assert hasattr(lib, name), name
    from paper_2402_06083_amd import msplit
    assert sorted(msplit.EXPORTED) == names


def test_struct_sizes_match_binding(lib, tmp_path):
    """Every field offset and struct size of the ctypes binding equals the C
    layout of include/msplit.h (compiled here with gcc)."""
    from paper_2402_06083_amd import msplit
    structs = {"msplit_options": msplit.Options, "msplit_roots": msplit.RootsC, "msplit_stats": msplit.Stats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "msplit.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'    printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'    printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                              check=True).stdout.split("\n") if line)
    for cname, py in structs.items():
        assert int(out[cname]) == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert int(out[f"{cname}.{fname}"]) == getattr(py, fname).offset, (cname, fname)


def test_header_constants_match_binding():
    from paper_2402_06083_amd import msplit
    text = open(HEADER).read()
    m = re.search(r"#define\s+MSPLIT_CERTIFY_WORKSPACE\s+(\d+)u?", text)
    assert m and int(m.group(1)) == msplit.CERTIFY_WORKSPACE
    m = re.search(r"#define\s+MSPLIT_STATIC_SCRATCH_BYTES\s+\((\d+)ull << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == msplit.STATIC_SCRATCH_BYTES
    for name, val in [("MSPLIT_R_REAL", msplit.R_REAL), ("MSPLIT_R_CERTIFIED", msplit.R_CERTIFIED),
                      ("MSPLIT_R_LABEL", msplit.R_LABEL), ("MSPLIT_R_DD", msplit.R_DD), ("MSPLIT_F_CERTIFY", msplit.F_CERTIFY),
                      ("MSPLIT_F_NO_LABEL", msplit.F_NO_LABEL), ("MSPLIT_F_BASIN", msplit.F_BASIN),
                      ("MSPLIT_F_SIMPLE", msplit.F_SIMPLE), ("MSPLIT_R_BASIN", msplit.R_BASIN),
                      ("MSPLIT_E_WORKSPACE", msplit.E_WORKSPACE), ("MSPLIT_F_CONJUGATES", msplit.F_CONJUGATES),
                      ("MSPLIT_DD", msplit.DD)]:
        m = re.search(name + r"\s*=\s*(-?\d+)u?", text)
        assert m and int(m.group(1)) == val, name


def test_expected_counts_match_oracle_counts(lib):
    from paper_2402_06083_amd import msplit
    for n in range(1, 31):
        assert msplit.expected_count(0, n) == 2 ** (n - 1)
        assert msplit.expected_count(0, n, True) == counts.hyp_count(n)
    for l in range(2, 12):
        for n in range(1, 12):
            assert msplit.expected_count(l, n) == counts.mis_count(l, n), (l, n)
    assert msplit.expected_count(1, 3) == 0
    assert msplit.expected_count(0, 0) == 0


def test_status_strings(lib):
    from paper_2402_06083_amd import msplit
    for code in range(0, -8, -1):
        s = msplit.strerror(code)
        assert s and s != "unknown status"
    assert msplit.strerror(-99) == "unknown status"


def test_invalid_arguments_without_device(lib):
    from paper_2402_06083_amd import msplit
    b = ctypes.c_uint64()
    L = msplit.lib()
    assert L.msplit_workspace_size(1, 3, None, ctypes.byref(b)) == msplit.E_ARG
    assert L.msplit_workspace_size(0, 0, None, ctypes.byref(b)) == msplit.E_ARG
    assert L.msplit_workspace_size(0, 31, None, ctypes.byref(b)) == msplit.E_ARG
    cnt = ctypes.c_uint64(7)
    assert L.msplit_hyperbolic(0, None, None, 0, None, ctypes.byref(cnt), None, None) == msplit.E_ARG
    assert cnt.value == 0
    assert L.msplit_misiurewicz(1, 3, None, None, 0, None, ctypes.byref(cnt), None, None) == msplit.E_ARG


def test_static_entry_point_limits_without_device(lib):
    """msplit_hyperbolic_static refuses, before any device work, a split
    whose workspace exceeds its static array (p_20 with the defaults), and
    null arguments; p_19 fits the array."""
    from paper_2402_06083_amd import msplit
    L = msplit.lib()
    assert msplit.workspace_size(0, 19, msplit.make_options(certify=True)) <= msplit.STATIC_SCRATCH_BYTES
    assert msplit.workspace_size(0, 20, msplit.make_options(certify=True)) > msplit.STATIC_SCRATCH_BYTES
    rs = msplit.RootsC(1, 1, None, None, None, None, None, None, 1, None)
    cnt = ctypes.c_uint64(7)
    assert L.msplit_hyperbolic_static(20, None, ctypes.byref(rs), ctypes.byref(cnt), None, None) == msplit.E_WORKSPACE
    assert cnt.value == 0
    assert L.msplit_hyperbolic_static(0, None, ctypes.byref(rs), ctypes.byref(cnt), None, None) == msplit.E_ARG
    assert L.msplit_hyperbolic_static(12, None, None, ctypes.byref(cnt), None, None) == msplit.E_ARG
