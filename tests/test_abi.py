"""The C-ABI library loads and exports every entry point declared in include/duq.h
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_1504_05708_amd import duq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names += re.findall(r"\b(duq_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = duq.lib()
    names = declared_functions()
    assert len(names) >= 8
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_header():
    assert set(duq.EXPORTS) == set(declared_functions())


def test_serve_threshold_matches_header():
    text = open(os.path.join(ROOT, "include", "duq.h")).read()
    m = re.search(r"#define DUQ_SERVE_BATCH_NMAX (\d+)", text)
    assert m and int(m.group(1)) == duq.SERVE_BATCH_NMAX


def test_default_options_and_strerror():
    o = duq.default_options()
    assert o.method == duq.DFGM and o.output == duq.LAST and o.eps_out == 1e-4 and o.eps_in == 1e-6
    assert o.safety == 1.02 and o.max_outer > 0 and o.serve_slice == 16
    assert duq.lib().duq_strerror(duq.DUQ_EINVAL) == b"invalid argument"


def test_struct_layout_matches_header(tmp_path):
    """Compile the header with the host C compiler and compare sizes/offsets
    with the ctypes mirrors."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    structs = {"duq_problem": duq.DuqProblem, "duq_options": duq.DuqOptions,
               "duq_result": duq.DuqResult, "duq_batch": duq.DuqBatch, "duq_request": duq.DuqRequest}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "duq.h"', 'int main(void){']
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
