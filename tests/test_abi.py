"""Host-side checks of the C ABI: the library loads and exports every
function declared in include/*.h.  No compute calls (no GPU here)."""

import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M):
            name = m.group(1)
            if name not in ("if", "while", "for", "return", "sizeof"):
                names.add(name)
    return names


def test_header_declares_the_entry_points():
    d = _declared()
    for name in ("mce_static", "imce_create", "imce_add_edges", "imce_destroy", "mce_strerror"):
        assert name in d


def test_library_exports_every_declared_symbol():
    import paper_2001_11433_amd as m
    L = m.lib()
    for name in sorted(_declared()):
        assert hasattr(L, name), name
    assert set(m.EXPORTS) <= _declared()


def test_strerror_names_every_code():
    import paper_2001_11433_amd as m
    L = m.lib()
    for code in (0, -1, -2, -3, -4, -5, -6):
        s = L.mce_strerror(code).decode()
        assert s and s != "unknown error"


def test_null_arguments_are_rejected_without_a_device():
    import paper_2001_11433_amd as m
    L = m.lib()
    assert L.mce_static(None, 0, None, None, None, None) == m.MCE_EINVAL
    assert L.mce_rank_metric(None, 0, None, None) == m.MCE_EINVAL


def test_oracle_and_library_share_no_code():
    # the two sides never import or include each other
    for path in glob.glob(os.path.join(ROOT, "paper_2001_11433_amd", "**", "*"), recursive=True):
        if os.path.isfile(path) and path.endswith((".py", ".hip", ".h", ".cpp")):
            txt = open(path).read()
            assert "oracle" not in re.findall(r"(?:import|include)\s+[\"<]?(\w+)", txt), path
    for path in glob.glob(os.path.join(ROOT, "oracle", "*")):
        if path.endswith((".py", ".cpp")):
            txt = open(path).read()
            assert "paper_2001_11433_amd" not in txt, path


def test_header_compiles_as_c99(tmp_path):
    # the boundary is a C ABI: a plain C caller must be able to use the header
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use.c"
    src.write_text(
        '#include "mce.h"\n'
        "int use(void) {\n"
        "  mce_csr g = {0};\n"
        "  mce_opts o = {0};\n"
        "  mce_result r;\n"
        "  imce_result b;\n"
        "  (void)b;\n"
        "  o.sched = MCE_SCHED_DEGREE;\n"
        "  return mce_static(&g, MCE_RANK_DEGENERACY, &o, &r, 0, 0) == MCE_OK ? 0 : 1;\n"
        "}\n")
    inc = os.path.join(ROOT, "include")
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-pedantic", "-fsyntax-only", "-I", inc, str(src)],
                   check=True)


def test_binding_structs_match_the_header(tmp_path):
    # sizes and field offsets of the public structs as a C compiler lays them
    # out, against the ctypes mirrors the binding passes through the ABI
    import shutil
    import subprocess
    import paper_2001_11433_amd as m
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"mce_opts": m._Opts, "mce_result": m._Result, "mce_clique_buf": m._CliqueBuf,
               "mce_per_vertex": m._PerVertex, "imce_result": m._ImceResult, "mce_csr": m._Csr}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mce.h"', "int main(void) {"]
    for cname, cty in structs.items():
        lines.append('  printf("%s %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in cty._fields_:
            lines.append('  printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                         check=True).stdout.splitlines())
    for cname, cty in structs.items():
        assert int(got[cname]) == ctypes.sizeof(cty), cname
        for fname, _ in cty._fields_:
            assert int(got["%s.%s" % (cname, fname)]) == getattr(cty, fname).offset, (cname, fname)
