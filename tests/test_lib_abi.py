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


def test_struct_layouts_match_header():
    from paper_2607_05929_amd import binding
    # sizes implied by the header's field order on LP64
    assert C.sizeof(binding.PlanDesc) == 4 * 3 + 4 + 8 + 4 * 18 + 4 * 2 + 8 * 2 + 4 + 4 + 8 + 4 * 5 + 4
    assert C.sizeof(binding.Material) == 8 + 8 * 8 + 8 * 4
    assert C.sizeof(binding.LoadStep) == 8 * (3 + 9 + 27) + 4 * 6 + 8 * 6 + 8
    assert C.sizeof(binding.IterEntry) == 4 * 2 + 8 + 4 * 2 + 8 * 6
