"""The C-ABI library: it builds, loads without a GPU, and exports every entry
point that include/qc.h declares.  No compute calls (CPU only)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s+\*?(qc_[a-z0-9_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("qc_solve_interval", "qc_apply_gains", "qc_residual", "qc_ctx_create", "qc_ctx_sync"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2412_10072_amd import qc
    if not os.path.exists(qc.LIB_PATH):
        pytest.skip("libqc.so not built")
    lib = qc.load_library()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"missing exports: {missing}"
    assert set(qc.EXPORTS) == set(declared_functions())


def test_binding_struct_layout_matches_header():
    """The ctypes structs mirror the C structs field for field (sizes of the
    C layout on x86-64 / LP64)."""
    import ctypes as C
    from paper_2412_10072_amd import qc
    assert C.sizeof(qc.QcVis) == 8 + 6 * 4 + 8 * 8
    assert qc.QcVis.data.offset == 32
    assert C.sizeof(qc.QcTerm) == 24 + 9 * 8
    assert qc.QcTerm.t_map.offset == 24
    assert C.sizeof(qc.QcSolveOpts) == 8 + 3 * 4 + 4 + 8 + 8
    assert C.sizeof(qc.QcSolveStats) == 5 * 8
    assert C.sizeof(qc.QcProblem) == C.sizeof(qc.QcVis) + C.sizeof(qc.QcTerm) + C.sizeof(qc.QcSolveStats) + 8


def test_binding_offsets_equal_the_c_compiler_s(tmp_path):
    """Every field offset and struct size of the ctypes mirrors equals what a C
    compiler gives for include/qc.h."""
    import ctypes as C
    import shutil
    import subprocess
    from paper_2412_10072_amd import qc
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"qc_vis": qc.QcVis, "qc_term": qc.QcTerm, "qc_solve_opts": qc.QcSolveOpts,
               "qc_solve_stats": qc.QcSolveStats, "qc_problem": qc.QcProblem, "qc_sky": qc.QcSky}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "qc.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "probe"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                        check=True).stdout.splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(py, fname).offset, f"{cname}.{fname}"


def test_context_without_device_fails_cleanly():
    import torch
    from paper_2412_10072_amd import qc
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    if not os.path.exists(qc.LIB_PATH):
        pytest.skip("libqc.so not built")
    with pytest.raises(qc.QcError):
        qc.Context(0)
