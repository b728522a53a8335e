"""ctypes binding of the catpc C ABI (include/catpc.h), same names as the C calls.

Argument marshalling only: every step of the hot path runs in the HIP library
(libcatpc.so, built by paper_1712_09430_amd/build.py).  If the library is not
built, loading raises; there is no fallback implementation.
"""
import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcatpc.so")

CATPC_OK = 0
CATPC_E_INVALID = -1
CATPC_E_CAPACITY = -2
CATPC_E_HIP = -3
CATPC_E_STATE = -5

FLAG_VALID, FLAG_STOP_SINPHI, FLAG_STOP_ARC, FLAG_SPD_FAIL, FLAG_REFIT64 = 1, 2, 4, 8, 16

N_STAGES = 8
STAGES = ("row_index", "grid", "neighbours", "clean_start", "scan", "compact", "tracklets", "refit64")

EXPORTS = ("catpc_track_batch_noalloc", "catpc_sector_frame", "catpc_to_global", "catpc_stage_times", "catpc_work_counts", "catpc_default_params", "catpc_default_tuning", "catpc_row_stride", "catpc_workspace_bytes", "catpc_create", "catpc_destroy",
           "catpc_set_params", "catpc_set_tuning", "catpc_get_tuning", "catpc_track_batch", "catpc_track_plain",
           "catpc_result", "catpc_fetch_tracklets", "catpc_select_tracklets", "catpc_select_result", "catpc_refit_tracks", "catpc_default_merge_params", "catpc_merge_tracks", "catpc_merge_counts", "catpc_fp32_probe", "catpc_phase_clocks", "catpc_probe_copy", "catpc_probe_fma",
           "catpc_last_error")


class CatpcError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"catpc status {status}: {message}")
        self.status = status


class catpc_params(ctypes.Structure):
    _fields_ = [("bz", ctypes.c_float), ("sigma_y", ctypes.c_float), ("sigma_z", ctypes.c_float),
                ("nf_win_y", ctypes.c_float), ("nf_win_z", ctypes.c_float), ("nf_chi2_max", ctypes.c_float),
                ("tc_gate_nsigma", ctypes.c_float), ("tc_max_miss", ctypes.c_int32), ("min_hits", ctypes.c_int32),
                ("precision", ctypes.c_int32)]


class catpc_geometry(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int32), ("row_x", ctypes.c_void_p), ("sectors_per_side", ctypes.c_int32)]


class catpc_tuning(ctypes.Structure):
    _fields_ = [("bin_hits", ctypes.c_float), ("nf_block", ctypes.c_int32), ("tc_block", ctypes.c_int32),
                ("tc_waves_per_cu", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("nf_rows", ctypes.c_int32), ("nf_lds_kb", ctypes.c_int32), ("tc_xcd", ctypes.c_int32),
                ("tc_occupancy", ctypes.c_int32), ("tc_sync", ctypes.c_int32),
                ("merge_pair_cap", ctypes.c_int32)]


_vp = ctypes.c_void_p


class catpc_input(ctypes.Structure):
    _fields_ = [("y", _vp), ("z", _vp), ("row", _vp), ("hit_offset", _vp), ("hit_offset_host", _vp),
                ("n_sectors", ctypes.c_int32), ("n_hits", ctypes.c_int64), ("x", _vp)]


class catpc_output(ctypes.Structure):
    _fields_ = [("link_up", _vp), ("link_dn", _vp), ("nf_up", _vp), ("nf_dn", _vp), ("start_hit", _vp),
                ("tracklet_offset", _vp), ("tracklet_capacity", ctypes.c_int64), ("x_ref", _vp), ("param", _vp),
                ("cov", _vp), ("row_hit", _vp), ("start_row", _vp), ("first_row", _vp), ("last_row", _vp),
                ("n_hits", _vp), ("flags", _vp)]


class catpc_fits(ctypes.Structure):
    _fields_ = [("x", _vp), ("param", _vp), ("cov", _vp), ("chi2", _vp), ("ndf", _vp), ("flags", _vp),
                ("capacity", ctypes.c_int64)]


class catpc_merge_params(ctypes.Structure):
    _fields_ = [("max_gap", ctypes.c_int32), ("window", ctypes.c_float), ("chi2_max", ctypes.c_float)]


class catpc_merges(ctypes.Structure):
    _fields_ = [("next", _vp), ("prev", _vp), ("head", _vp), ("chi2", _vp), ("capacity", ctypes.c_int64)]


class catpc_tracks(ctypes.Structure):
    _fields_ = [("track_offset", _vp), ("track_tracklet", _vp), ("track_n_hits", _vp), ("track_hit_offset", _vp),
                ("track_capacity", ctypes.c_int64), ("track_hits", _vp), ("hit_capacity", ctypes.c_int64)]


_lib = None


def use_library(path):
    """Bind the functions below to another build of the library (the
    profiling build, `build.PHASE_LIB`); the next call loads it.  Contexts
    made with the previous library must be destroyed first."""
    global _lib, LIB_PATH
    LIB_PATH = path
    _lib = None


def lib():
    """Load libcatpc.so; raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        # torch first: its libraries load the HIP runtime bundled with them
        # under the unversioned name, which a runtime loaded earlier under its
        # versioned name (the library's own dependency) does not satisfy.  Two
        # HIP runtimes in one process do not share the device (the second one
        # reports none), so the library must bind to torch's, already loaded.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        st = ctypes.c_int32
        P = ctypes.POINTER
        L.catpc_default_params.argtypes = [P(catpc_params)]
        L.catpc_default_params.restype = None
        L.catpc_default_tuning.argtypes = [P(catpc_tuning)]
        L.catpc_default_tuning.restype = None
        L.catpc_row_stride.argtypes = [ctypes.c_int32]
        L.catpc_row_stride.restype = ctypes.c_int32
        L.catpc_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32]
        L.catpc_workspace_bytes.restype = ctypes.c_size_t
        L.catpc_create.argtypes = [P(catpc_geometry), P(catpc_params), ctypes.c_int64, ctypes.c_int32, P(_vp)]
        L.catpc_track_batch_noalloc.argtypes = [ctypes.c_int32, _vp, P(catpc_params), P(catpc_tuning), _vp, _vp,
                                                 _vp, _vp]
        L.catpc_track_batch_noalloc.restype = st
        L.catpc_sector_frame.argtypes = [P(catpc_geometry), ctypes.c_int32, P(ctypes.c_double), P(ctypes.c_int32)]
        L.catpc_sector_frame.restype = st
        L.catpc_to_global.argtypes = [P(catpc_geometry), ctypes.c_int32, ctypes.c_int64, _vp, _vp, _vp]
        L.catpc_to_global.restype = st
        L.catpc_create.restype = st
        L.catpc_destroy.argtypes = [_vp]
        L.catpc_destroy.restype = None
        L.catpc_set_params.argtypes = [_vp, P(catpc_params)]
        L.catpc_set_params.restype = st
        L.catpc_set_tuning.argtypes = [_vp, P(catpc_tuning)]
        L.catpc_set_tuning.restype = st
        L.catpc_get_tuning.argtypes = [_vp, P(catpc_tuning)]
        L.catpc_get_tuning.restype = st
        for f in ("catpc_track_batch", "catpc_track_plain"):
            getattr(L, f).argtypes = [_vp, P(catpc_input), P(catpc_output), _vp]
            getattr(L, f).restype = st
        L.catpc_result.argtypes = [_vp, _vp, P(ctypes.c_int64)]
        L.catpc_result.restype = st
        L.catpc_fetch_tracklets.argtypes = [_vp, P(catpc_input), ctypes.c_int64, P(catpc_output), _vp]
        L.catpc_fetch_tracklets.restype = st
        L.catpc_select_tracklets.argtypes = [_vp, P(catpc_input), P(catpc_output), P(catpc_tracks), _vp]
        L.catpc_select_tracklets.restype = st
        L.catpc_select_result.argtypes = [_vp, _vp, P(ctypes.c_int64), P(ctypes.c_int64)]
        L.catpc_refit_tracks.argtypes = [_vp, P(catpc_input), P(catpc_output), P(catpc_tracks), P(catpc_fits), _vp]
        L.catpc_refit_tracks.restype = st
        L.catpc_default_merge_params.argtypes = [P(catpc_merge_params)]
        L.catpc_default_merge_params.restype = None
        L.catpc_merge_tracks.argtypes = [_vp, P(catpc_input), P(catpc_output), P(catpc_tracks), P(catpc_fits),
                                         P(catpc_merge_params), P(catpc_merges), _vp]
        L.catpc_merge_tracks.restype = st
        L.catpc_merge_counts.argtypes = [_vp, _vp, P(ctypes.c_int64), P(ctypes.c_int64)]
        L.catpc_merge_counts.restype = st
        L.catpc_select_result.restype = st
        L.catpc_stage_times.argtypes = [_vp, P(catpc_input), P(catpc_output), _vp, _vp]
        L.catpc_stage_times.restype = st
        L.catpc_work_counts.argtypes = [_vp, _vp, _vp]
        L.catpc_work_counts.restype = st
        L.catpc_fp32_probe.argtypes = [ctypes.c_int32, _vp, _vp, _vp, ctypes.c_int64, _vp]
        L.catpc_fp32_probe.restype = st
        L.catpc_phase_clocks.argtypes = [P(ctypes.c_uint64), ctypes.c_int32]
        L.catpc_phase_clocks.restype = st
        L.catpc_probe_copy.argtypes = [_vp, _vp, ctypes.c_int64, _vp]
        L.catpc_probe_copy.restype = st
        L.catpc_probe_fma.argtypes = [_vp, ctypes.c_int64, ctypes.c_int32, _vp]
        L.catpc_probe_fma.restype = st
        L.catpc_last_error.argtypes = []
        L.catpc_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def catpc_last_error():
    return lib().catpc_last_error().decode()


def _check(status, allow=()):
    if status != CATPC_OK and status not in allow:
        raise CatpcError(status, catpc_last_error())
    return status


def catpc_default_params():
    p = catpc_params()
    lib().catpc_default_params(ctypes.byref(p))
    return p


def catpc_default_tuning():
    t = catpc_tuning()
    lib().catpc_default_tuning(ctypes.byref(t))
    return t


def catpc_default_merge_params():
    m = catpc_merge_params()
    lib().catpc_default_merge_params(ctypes.byref(m))
    return m


def catpc_row_stride(n_rows):
    return int(lib().catpc_row_stride(n_rows))


def catpc_workspace_bytes(n_rows, max_hits, max_sectors):
    return int(lib().catpc_workspace_bytes(n_rows, max_hits, max_sectors))


def catpc_geometry_of(row_x, sectors_per_side=18):
    """A catpc_geometry for row_x (the array is kept on the returned struct)."""
    rx = np.ascontiguousarray(row_x, np.float32)
    g = catpc_geometry(len(rx), rx.ctypes.data, int(sectors_per_side))
    g._rx = rx
    return g


def catpc_create(row_x, params, max_hits, max_sectors, sectors_per_side=18):
    g = catpc_geometry_of(row_x, sectors_per_side)
    h = _vp()
    _check(lib().catpc_create(ctypes.byref(g), ctypes.byref(params), int(max_hits), int(max_sectors),
                              ctypes.byref(h)))
    return h


def catpc_track_batch_noalloc(n_rows, row_x_dev, params, tuning, inp, out, status_dev, stream):
    """The batched chain on the library's fixed workspace (no allocation);
    row_x_dev and status_dev are device addresses, tuning may be None."""
    _check(lib().catpc_track_batch_noalloc(int(n_rows), row_x_dev, ctypes.byref(params),
                                           ctypes.byref(tuning) if tuning is not None else None,
                                           ctypes.byref(inp), ctypes.byref(out), status_dev, stream))


def catpc_sector_frame(geom, sector_id):
    """(alpha rad, side +1/-1) of a sector (host call)."""
    a, sd = ctypes.c_double(), ctypes.c_int32()
    _check(lib().catpc_sector_frame(ctypes.byref(geom), int(sector_id), ctypes.byref(a), ctypes.byref(sd)))
    return a.value, sd.value


def catpc_to_global(geom, sector_id, x, param):
    """Sector-frame (x, y, z, sin phi, tan lambda, q/pT) -> global (X, Y, Z,
    phi, tan lambda, q/pT), float64[n, 6] (host call)."""
    xs = np.ascontiguousarray(x, np.float32)
    ps = np.ascontiguousarray(param, np.float32).reshape(-1, 5)
    out = np.empty((len(xs), 6), np.float64)
    _check(lib().catpc_to_global(ctypes.byref(geom), int(sector_id), len(xs), xs.ctypes.data, ps.ctypes.data,
                                 out.ctypes.data))
    return out


def catpc_destroy(ctx):
    lib().catpc_destroy(ctx)


def catpc_set_params(ctx, params):
    _check(lib().catpc_set_params(ctx, ctypes.byref(params)))


def catpc_set_tuning(ctx, tuning):
    _check(lib().catpc_set_tuning(ctx, ctypes.byref(tuning)))


def catpc_get_tuning(ctx):
    t = catpc_tuning()
    _check(lib().catpc_get_tuning(ctx, ctypes.byref(t)))
    return t


def catpc_track_batch(ctx, inp, out, stream):
    return _check(lib().catpc_track_batch(ctx, ctypes.byref(inp), ctypes.byref(out), stream))


def catpc_track_plain(ctx, inp, out, stream):
    return _check(lib().catpc_track_plain(ctx, ctypes.byref(inp), ctypes.byref(out), stream))


def catpc_result(ctx, stream):
    """Synchronise; returns (status, n_tracklets).  CATPC_E_CAPACITY is returned,
    not raised (fetch the rest with catpc_fetch_tracklets)."""
    n = ctypes.c_int64(0)
    st = _check(lib().catpc_result(ctx, stream, ctypes.byref(n)), allow=(CATPC_E_CAPACITY,))
    return st, int(n.value)


def catpc_fetch_tracklets(ctx, inp, first, out, stream):
    return _check(lib().catpc_fetch_tracklets(ctx, ctypes.byref(inp), int(first), ctypes.byref(out), stream))


def catpc_select_tracklets(ctx, inp, trk, tracks, stream):
    return _check(lib().catpc_select_tracklets(ctx, ctypes.byref(inp), ctypes.byref(trk), ctypes.byref(tracks),
                                               stream))


def catpc_refit_tracks(ctx, inp, trk, tracks, fits, stream):
    return _check(lib().catpc_refit_tracks(ctx, ctypes.byref(inp), ctypes.byref(trk), ctypes.byref(tracks),
                                           ctypes.byref(fits), stream))


def catpc_merge_counts(ctx, stream):
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().catpc_merge_counts(ctx, stream, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def catpc_merge_tracks(ctx, inp, trk, tracks, fits, mp, out, stream):
    return _check(lib().catpc_merge_tracks(ctx, ctypes.byref(inp), ctypes.byref(trk), ctypes.byref(tracks),
                                           ctypes.byref(fits), None if mp is None else ctypes.byref(mp),
                                           ctypes.byref(out), stream))


def catpc_select_result(ctx, stream):
    """Synchronise; returns (n_tracks, n_track_hits) of the last selection."""
    nt, nh = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib().catpc_select_result(ctx, stream, ctypes.byref(nt), ctypes.byref(nh)))
    return int(nt.value), int(nh.value)


def catpc_stage_times(ctx, inp, out, stream):
    """Per-stage milliseconds (numpy float32[N_STAGES]) of one batched run."""
    ms = np.zeros(N_STAGES, np.float32)
    _check(lib().catpc_stage_times(ctx, ctypes.byref(inp), ctypes.byref(out), stream, ms.ctypes.data))
    return ms


def catpc_work_counts(ctx, stream):
    """[transports, updates, gated candidates, row searches] of the last call."""
    c = np.zeros(4, np.int64)
    _check(lib().catpc_work_counts(ctx, stream, c.ctypes.data))
    return c


def catpc_fp32_probe(op, a, b, out, n, stream):
    return _check(lib().catpc_fp32_probe(int(op), a, b, out, int(n), stream))


PHASE_SLOTS = 9


def catpc_phase_clocks(clear=False):
    """Phase clocks of a profiling build (see include/catpc.h); a list of
    PHASE_SLOTS ints, or None after a clear."""
    buf = (ctypes.c_uint64 * PHASE_SLOTS)()
    _check(lib().catpc_phase_clocks(buf, 1 if clear else 0))
    return None if clear else [int(v) for v in buf]


def catpc_probe_copy(src, dst, n_bytes, stream):
    return _check(lib().catpc_probe_copy(src, dst, int(n_bytes), stream))


def catpc_probe_fma(out, n_threads, n_iter, stream):
    return _check(lib().catpc_probe_fma(out, int(n_threads), int(n_iter), stream))
