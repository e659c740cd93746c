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


def test_descriptor_tables_match_field_by_field_filling():
    """The binding fills its call descriptors as u64 tables; every field must
    equal what setting the ctypes fields one by one gives (CPU tensors stand in
    for device ones: only addresses and sizes are read)."""
    torch = pytest.importorskip("torch")
    F = 3
    frames = [torch.empty((F, 1000 + 7 * j)) for j in range(5)]
    methods = [lcp.METHOD_AUTO, lcp.METHOD_S, lcp.METHOD_T, lcp.METHOD_S, lcp.METHOD_AUTO]
    arr, _tab = lcp.frame_in_table(frames, F, methods)
    for j, f in enumerate(frames):
        assert [arr[j].fields[k] for k in range(F)] == [f[k].data_ptr() for k in range(F)]
        assert all(not arr[j].fields[k] for k in range(F, lcp.MAX_FIELDS))
        assert arr[j].n == f.shape[1] and arr[j].method == methods[j]
    arr, _tab = lcp.frame_in_table(frames[:2], F)
    assert arr[1].method == lcp.METHOD_AUTO
    buf = torch.empty(1000, dtype=torch.uint8)
    offsets = [0, 100, 250, 400, 401, 999]
    blobs, _b = lcp.blob_table(buf.data_ptr(), offsets)
    for j in range(5):
        assert blobs[j].data == buf.data_ptr() + offsets[j]
        assert blobs[j].size == offsets[j + 1] - offsets[j]
    blobs, _b = lcp.blob_table(buf.data_ptr(), offsets, sizes=[5, 6, 7, 8, 9])
    assert [blobs[j].size for j in range(5)] == [5, 6, 7, 8, 9]
    outs = [torch.empty((F, 2000))[:, : 1500 + j] for j in range(4)]  # row stride 2000
    fo, _o = lcp.frame_out_table(outs, F)
    for j, o in enumerate(outs):
        assert [fo[j].fields[k] for k in range(F)] == [o[k].data_ptr() for k in range(F)]
        assert fo[j].capacity == o.shape[1]


def test_static_entry_refuses_on_the_host():
    """lcp_compress_static checks its parameters and whether the scratch they
    need fits its static array before any HIP call, so the refusals show on a
    machine without a GPU too."""
    import ctypes as C
    if not os.path.exists(lcp.LIB_PATH):
        pytest.skip("library not built")
    L = lcp.lib()

    def call(n, multi=0, k=4, frames=0, F=3):
        p = lcp.lcp_params(lcp.EB_ABS, 1e-3, F, multi, 0, k, 10, n, 0, 0, 0, frames)
        offs = (C.c_uint64 * 2)()
        return L.lcp_compress_static(C.byref(p), 0, None, None, 0, offs, None, None)

    assert call(1 << 20) == lcp.ERR_BUDGET          # 2^20 particles need more than 64 MiB
    assert call(500000) != lcp.ERR_BUDGET           # about 550,000 three-field particles fit
    assert call(600000) == lcp.ERR_BUDGET
    assert call(340000, F=6) != lcp.ERR_BUDGET      # about 370,000 of six fields
    assert call(400000, F=6) == lcp.ERR_BUDGET
    assert call(1000, frames=64) == lcp.ERR_BUDGET  # 64 frames per launch set
    assert call(1000, multi=1) == lcp.ERR_ARG       # LCP-S only
    assert call(1000, k=-1) == lcp.ERR_ARG          # no block-size search
    assert call(0) == lcp.ERR_ARG
