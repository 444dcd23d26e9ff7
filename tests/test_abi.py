"""The C-ABI library loads on a machine without a GPU, exports every function
include/gj.h declares, and validates join graphs on the host."""
import os
import re
import subprocess

import pytest

from conftest import ROOT


def _declared():
    src = open(os.path.join(ROOT, "include", "gj.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(gj_[a-z_0-9]+)\s*\(", src))
    # drop typedef'd function-pointer types
    return sorted(n for n in names if not n.endswith("_fn"))


def test_library_exports_every_declared_function():
    from paper_2206_10435_amd import gj

    lib = os.path.join(ROOT, "paper_2206_10435_amd", "libgj.so")
    assert os.path.exists(lib), "build libgj.so first"
    out = subprocess.run(["nm", "-D", "--defined-only", lib], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (gj_\w+)", out))
    declared = _declared()
    assert len(declared) >= 20
    missing = [n for n in declared if n not in exported]
    assert not missing, missing
    # and the binding knows the signature of each
    assert set(declared) <= set(gj.SIGNATURES), set(declared) - set(gj.SIGNATURES)
    gj.load_library()


def test_validate_graphs():
    from paper_2206_10435_amd import gj

    gj.validate([5, 5, 5], [2, 2, 2], [-1, 0, 1], [0, 0, 0], [0, 1, 1])
    bad = [
        ([5, 5], [2, 2], [-1, 1], [0, 0], [0, 1], gj.GJ_E_GRAPH),      # parent not earlier
        ([5, 5], [2, 2], [0, 0], [0, 0], [0, 1], gj.GJ_E_GRAPH),       # root has a parent
        ([5, 5], [2, 2], [-1, 0], [0, 2], [0, 1], gj.GJ_E_GRAPH),      # separator column out of range
        ([5, 5], [2, 2], [-1, 0], [0, 0], [0, 3], gj.GJ_E_GRAPH),      # parent column out of range
        ([5, 5], [0, 2], [-1, 0], [0, 0], [0, 0], gj.GJ_E_INVALID),    # no key columns
        ([5, 5], [9, 2], [-1, 0], [0, 0], [0, 1], gj.GJ_E_INVALID),    # too many key columns
        ([-1, 5], [2, 2], [-1, 0], [0, 0], [0, 1], gj.GJ_E_INVALID),   # negative size
        ([2**31, 5], [2, 2], [-1, 0], [0, 0], [0, 1], gj.GJ_E_INVALID),  # row ids beyond int32
    ]
    for rows, keys, par, sep, pcol, code in bad:
        with pytest.raises(gj.GJError) as ei:
            gj.validate(rows, keys, par, sep, pcol)
        assert ei.value.status == code, (rows, keys, par, sep, pcol)
    # more children than supported
    n = 10
    with pytest.raises(gj.GJError) as ei:
        gj.validate([3] * n, [1] + [1] * (n - 1), [-1] + [0] * (n - 1), [0] * n, [0] * n)
    assert ei.value.status == gj.GJ_E_GRAPH
    with pytest.raises(gj.GJError):
        gj.validate([3] * 17, [2] * 17, [-1] + list(range(16)), [0] * 17, [0] + [1] * 16)
