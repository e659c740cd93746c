"""CPU checks of the C ABI library: it loads without a GPU and exports every
function include/lcp.h declares; status strings are defined."""
import os
import re
import subprocess

import pytest

from paper_2411_00761_amd import lcp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lcp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lcp_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(lcp.LIB_PATH):
        pytest.skip("library not built")
    names = declared_functions()
    assert len(names) >= 10
    out = subprocess.run(["nm", "-D", "--defined-only", lcp.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (lcp_\w+)", out))
    assert set(names) <= exported, set(names) - exported
    assert set(lcp.EXPORTED) == set(names)
    L = lcp.lib()
    for n in names:
        assert hasattr(L, n)


def test_status_strings():
    if not os.path.exists(lcp.LIB_PATH):
        pytest.skip("library not built")
    L = lcp.lib()
    for st in range(9):
        assert L.lcp_status_string(st)
    assert L.lcp_status_string(4) == b"output buffer too small"
