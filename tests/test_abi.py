"""The C-ABI library loads and exports every symbol include/catpc.h declares;
host-side argument validation (no GPU needed: every call below fails before
touching the device)."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_1712_09430_amd.build as B
from paper_1712_09430_amd import catpc as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    text = open(os.path.join(ROOT, "include", "catpc.h")).read()
    return sorted(set(re.findall(r"\b(catpc_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    B.build(force=False)
    return C.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(C.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (catpc_\w+)", out))
    assert exported == set(names)


def test_defaults(lib):
    p = C.catpc_default_params()
    assert (p.bz, p.tc_max_miss, p.min_hits, p.precision) == (pytest.approx(0.5), 4, 10, 0)
    t = C.catpc_default_tuning()
    assert t.nf_block == 256 and t.use_graph == 1


def test_workspace_scales_linearly(lib):
    a = C.catpc_workspace_bytes(159, 1_000_000, 36)
    b = C.catpc_workspace_bytes(159, 2_000_000, 36)
    c = C.catpc_workspace_bytes(159, 3_000_000, 36)
    assert a > 0 and abs((c - b) - (b - a)) < 4096
    assert C.catpc_workspace_bytes(2, 10, 1) == 0


def test_host_validation(lib):
    p = C.catpc_default_params()
    with pytest.raises(C.CatpcError) as e:
        C.catpc_create([85.0, 84.0, 86.0], p, 10, 1)
    assert e.value.status == C.CATPC_E_INVALID and "ascending" in C.catpc_last_error()
    bad = C.catpc_default_params()
    bad.precision = 3
    with pytest.raises(C.CatpcError):
        C.catpc_create([85.0, 86.0, 87.0], bad, 10, 1)
    with pytest.raises(C.CatpcError):
        C.catpc_create([85.0, 86.0, 87.0], p, 1 << 31, 1)
    assert lib.catpc_track_batch(None, None, None, None) == C.CATPC_E_INVALID
    assert lib.catpc_result(None, None, None) == C.CATPC_E_INVALID
    assert lib.catpc_fp32_probe(7, None, None, None, 1, None) == C.CATPC_E_INVALID


def test_row_stride(lib):
    assert [C.catpc_row_stride(n) for n in (1, 7, 8, 9, 159, 160)] == [8, 8, 8, 16, 160, 160]
    assert C.catpc_row_stride(0) == 0
