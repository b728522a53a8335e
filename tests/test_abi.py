"""The C-ABI library loads and exports every symbol include/catpc.h declares;
host-side argument validation (no GPU needed: every call below fails before
touching the device)."""
import ctypes
import json
import os
import re
import subprocess
import sys

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
    # the product build records no phase clocks (only the profiling build does)
    assert lib.catpc_phase_clocks(None, 1) == C.CATPC_E_INVALID
    assert "profiling build" in C.catpc_last_error()


def test_row_stride(lib):
    assert [C.catpc_row_stride(n) for n in (1, 7, 8, 9, 159, 160)] == [8, 8, 8, 16, 160, 160]
    assert C.catpc_row_stride(0) == 0


def test_sector_frames_follow_the_generator(lib):
    """catpc_sector_frame agrees with the event generator's own sector
    rotations (2 x 18 sectors, Sec. 2) and sides."""
    import synth
    g = C.catpc_geometry_of(synth.row_x())
    for s in range(36):
        a, side = C.catpc_sector_frame(g, s)
        assert a == pytest.approx(synth.sector_alpha(s), abs=1e-12)
        assert side == (1 if s < 18 else -1)
    for s in (-1, 36):
        with pytest.raises(C.CatpcError):
            C.catpc_sector_frame(g, s)


def test_to_global_matches_the_closed_form_helix(lib):
    """Sector-frame parameters of generator helices (closed form, evaluated
    in the sector's rotated frame) map to the same helix evaluated in the
    global frame: position, momentum azimuth (also from a finite difference
    along the helix), dip and curvature."""
    import math

    import numpy as np

    import synth
    g = C.catpc_geometry_of(synth.row_x())
    # (q/pT, tan lambda, launch angle from the sector's centre, sector, path):
    # tracks leaving the origin through their sector, as the tracker sees them
    cases = [(1.0 / 0.5, 0.3, 0.05, 5, 120.0), (-1.0 / 2.0, -0.8, -0.1, 23, 200.0), (1.0 / 8.0, 0.0, 0.12, 17, 90.0),
             (-1.0 / 0.3, 1.0, -0.02, 30, 150.0)]
    for qpt, tanl, dphi, s, path in cases:
        a = synth.sector_alpha(s)
        phi0 = a + dphi
        x, y, z, sp = synth.helix_point(qpt, tanl, phi0, synth.BZ, a, path)
        X, Y, Z, SP = synth.helix_point(qpt, tanl, phi0, synth.BZ, 0.0, path)
        o = C.catpc_to_global(g, s, [x], [[y, z, sp, tanl, qpt]])[0]
        tol = 4e-5 * max(1.0, abs(x), abs(y), abs(z))  # binary32 inputs
        assert o[0] == pytest.approx(X, abs=tol) and o[1] == pytest.approx(Y, abs=tol)
        assert o[2] == pytest.approx(Z, abs=tol)
        assert math.sin(o[3]) == pytest.approx(SP, abs=1e-6)
        p1 = synth.helix_point(qpt, tanl, phi0, synth.BZ, 0.0, path + 1e-4)
        p0 = synth.helix_point(qpt, tanl, phi0, synth.BZ, 0.0, path - 1e-4)
        d = math.atan2(p1[1] - p0[1], p1[0] - p0[0])
        assert math.remainder(o[3] - d, 2 * math.pi) == pytest.approx(0.0, abs=1e-6)
        assert -math.pi < o[3] <= math.pi
        assert o[4] == np.float32(tanl) and o[5] == np.float32(qpt)
    with pytest.raises(C.CatpcError):
        C.catpc_to_global(g, 0, [100.0], [[0.0, 0.0, 1.5, 0.0, 0.0]])


def test_no_alloc_entry_point_validates_on_the_host(lib):
    """catpc_track_batch_noalloc rejects, before touching the device, an input
    beyond its fixed workspace and calls without a status word (host arrays
    stand in for the device pointers: nothing is enqueued)."""
    import numpy as np
    rx = np.arange(85.0, 85.0 + 159.0, dtype=np.float32)
    word = np.zeros(1, np.uint64)
    inp, out = C.catpc_input(), C.catpc_output()
    inp.n_sectors, inp.n_hits = 36, 3_000_000
    p = C.catpc_default_params()
    with pytest.raises(C.CatpcError) as e:
        C.catpc_track_batch_noalloc(159, rx.ctypes.data, p, None, inp, out, word.ctypes.data, None)
    assert e.value.status == C.CATPC_E_INVALID and "fixed workspace" in C.catpc_last_error()
    inp.n_hits = 1000
    with pytest.raises(C.CatpcError) as e:
        C.catpc_track_batch_noalloc(159, rx.ctypes.data, p, None, inp, out, None, None)
    assert "status" in C.catpc_last_error()
    bad = C.catpc_default_tuning()
    bad.nf_block = 1024
    with pytest.raises(C.CatpcError):
        C.catpc_track_batch_noalloc(159, rx.ctypes.data, p, bad, inp, out, word.ctypes.data, None)


def test_one_hip_runtime_when_the_library_loads_first():
    """Loading the library before anything imports torch still leaves one
    HIP runtime in the process (torch's): a second runtime would not see the
    device.  Checked in a fresh process, from its memory map."""
    code = ("import json, os, sys; sys.path.insert(0, %r)\n"
            "from paper_1712_09430_amd import catpc as C\n"
            "C.lib()\n"
            "import torch\n"
            "m = open('/proc/%%d/maps' %% os.getpid()).read().splitlines()\n"
            "print(json.dumps(sorted(set(l.split()[-1] for l in m if 'libamdhip64' in l))))\n") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    libs = json.loads(out.stdout.strip().splitlines()[-1])
    assert len(libs) == 1, libs
