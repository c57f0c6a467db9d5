"""The C-ABI library loads and exports every symbol its header declares
(no compute calls: these run without a GPU)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rjpath.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rjpath_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for need in ("rjpath_init_medium", "rjpath_run_chains", "rjpath_intensity", "rjpath_grad",
                 "rjpath_free_medium", "rjpath_last_error"):
        assert need in names


def test_library_exports_every_declared_symbol():
    from paper_1811_04156_amd import rjpath
    lib = rjpath.load()
    for name in declared():
        assert hasattr(lib, name), name
    assert lib.rjpath_version().decode().startswith("rjpath")


def test_python_binding_covers_the_header():
    from paper_1811_04156_amd import rjpath
    assert set(declared()) == set(rjpath.EXPORTS)


def test_missing_library_fails_loudly(tmp_path):
    from paper_1811_04156_amd import rjpath
    old = rjpath._lib
    rjpath._lib = None
    try:
        with pytest.raises(RuntimeError, match="missing"):
            rjpath.load(str(tmp_path / "nope.so"))
    finally:
        rjpath._lib = old


def test_struct_layouts_match_the_header(tmp_path):
    """Every field offset and struct size of the ctypes mirrors equals the C
    compiler's for the header."""
    import ctypes as C
    import subprocess
    from paper_1811_04156_amd import rjpath
    structs = {"rjpath_medium_desc": rjpath.MediumDesc, "rjpath_targets": rjpath.Targets,
               "rjpath_chains": rjpath.Chains, "rjpath_run_params": rjpath.RunParams}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for l in out:
        if l.strip():
            a, b, c = l.split()
            got[(a, b)] = int(c)
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
