"""CPU-side checks of the C ABI: the library loads, exports every function
declared in include/fmsolve.h, and validates descriptors without a GPU
(fm_workspace_bytes makes no device call)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "fmsolve.h")


def _declared():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fm_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2607_05929_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        # nothing built yet: compile it (hipcc cross-compiles gfx950 without a GPU)
        from paper_2607_05929_amd import build as _b
        _b.build()
    return binding.lib()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    from paper_2607_05929_amd import binding
    assert set(names) == set(binding.EXPORTS), set(names) ^ set(binding.EXPORTS)


def test_workspace_bytes_and_validation(lib):
    from paper_2607_05929_amd import binding
    p = W.config_inclusion32()
    d = binding.plan_desc(p)
    nb = lib.fm_workspace_bytes(C.byref(d))
    n = 33 ** 3
    assert nb > 3 * n * 8 * (1 + 2 * p.aa_depth)      # u^f + two FP64 rings at least
    d32 = binding.plan_desc(p, prec=W.FP32_MIXED)
    assert lib.fm_workspace_bytes(C.byref(d32)) < nb
    # periodic on one face only is rejected
    bad = binding.plan_desc(p)
    bad.bc[0 * 6 + 1 * 2 + 0] = W.P
    bad.bc[0 * 6 + 1 * 2 + 1] = W.D
    assert lib.fm_workspace_bytes(C.byref(bad)) == 0
    assert b"periodic" in lib.fm_last_error()
    bad2 = binding.plan_desc(p)
    bad2.aa_depth = 9
    assert lib.fm_workspace_bytes(C.byref(bad2)) == 0
    bad3 = binding.plan_desc(p)
    bad3.n[1] = 1
    assert lib.fm_workspace_bytes(C.byref(bad3)) == 0


def _c_layout(structs):
    """Field offsets and sizes of header structs, from a C program compiled
    against include/fmsolve.h with the host compiler."""
    import shutil
    import subprocess
    import tempfile
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "fmsolve.h"', "int main(void) {"]
    for cname, fields in structs:
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in fields:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        with open(src, "w") as f:
            f.write("\n".join(lines))
        subprocess.run([cc, "-I", os.path.join(ROOT, "include"), "-o", exe, src], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    res = {}
    for ln in out.splitlines():
        cname, field, val = ln.split()
        res[(cname, field)] = int(val)
    return res


def test_struct_layouts_match_header():
    """Every ctypes mirror in the binding has the header's field offsets and size."""
    from paper_2607_05929_amd import binding as B
    pairs = [("fm_plan_desc", B.PlanDesc), ("fm_material", B.Material), ("fm_load_step", B.LoadStep),
             ("fm_outputs", B.Outputs), ("fm_iter_entry", B.IterEntry), ("fm_iter_log", B.IterLog),
             ("fm_request", B.Request), ("fm_stats", B.Stats)]
    lay = _c_layout([(c, [f for f, _ in py._fields_]) for c, py in pairs])
    for cname, py in pairs:
        assert lay[(cname, "size")] == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert lay[(cname, f)] == getattr(py, f).offset, (cname, f)
