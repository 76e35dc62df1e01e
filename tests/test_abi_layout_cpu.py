"""The ctypes mirrors of the C ABI's structs (paper_2508_05958_amd/__init__.py)
against include/htlr.h: a small C program compiled with the host compiler
prints sizeof and offsetof of every field, and each mirror must agree field by
field (name order, offset, total size).  Catches a field added on one side
only, which would shift every later field across the boundary."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.join(os.path.dirname(__file__), "..")
HEADER = os.path.join(ROOT, "include", "htlr.h")

PAIRS = {
    "htlr_build_opts": "_BuildOpts",
    "htlr_solve_opts": "_SolveOpts",
    "htlr_solve_info": "_SolveInfo",
    "htlr_info_t": "_Info",
    "htlr_tune_result": "_TuneResult",
    "htlr_profile_entry": "_ProfEntry",
    "htlr_server_opts": "_ServerOpts",
    "htlr_request": "_Request",
    "htlr_request_info": "_RequestInfo",
    "htlr_server_stats_t": "_ServerStats",
}


def _c_fields(src, name):
    """Field names of 'typedef struct { ... } name;' in declaration order."""
    end = re.search(r"\}\s*" + re.escape(name) + r"\s*;", src)
    assert end, name
    start = src.rfind("typedef struct {", 0, end.start())
    body = re.sub(r"/\*.*?\*/", "", src[start + len("typedef struct {"):end.start()], flags=re.S)
    out = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        # "type a, b[16], *c" -> a, b, c: the first declarator follows the type
        parts = decl.split(",")
        for k, part in enumerate(parts):
            tok = part.strip().split()[-1] if k == 0 else part.strip()
            out.append(re.sub(r"\[.*\]", "", tok.lstrip("*")))
    return out


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    src = open(HEADER).read()
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "htlr.h"', "int main(void) {"]
    for cname in PAIRS:
        lines.append(f'  printf("%s size %zu\\n", "{cname}", sizeof({cname}));')
        for f in _c_fields(src, cname):
            lines.append(f'  printf("%s %s %zu\\n", "{cname}", "{f}", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    d = tmp_path_factory.mktemp("abi")
    c = d / "layout.c"
    c.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    res = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        s, f, v = line.split()
        res.setdefault(s, {})[f] = int(v)
    return res


@pytest.mark.parametrize("cname", sorted(PAIRS))
def test_ctypes_mirror_matches_header(c_layout, cname):
    import ctypes
    import paper_2508_05958_amd as H
    py = getattr(H, PAIRS[cname])
    want = c_layout[cname]
    names = [f for f in want if f != "size"]
    assert [n for n, _ in py._fields_] == names
    for n, _ in py._fields_:
        assert getattr(py, n).offset == want[n], (cname, n)
    assert ctypes.sizeof(py) == want["size"]
