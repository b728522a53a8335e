"""CPU oracle for the sector-tracking hot path -- TEST INFRASTRUCTURE.

Only tests/, __graft_entry__.smoke() and the cpu_baseline leg of bench.py may
import this package.  The product (paper_1712_09430_amd) never does: it shares
no code, header, table or helper with the oracle.

The arithmetic lives in plain C (tracker.c, links.c, refit_mixed.c), built by
oracle/build.py; this module only marshals numpy arrays through ctypes.  All
functions work on one sector (sector-local, row-sorted hits).  Modes: "f32"
(every operation rounded to binary32, the precision whose decisions the GPU
path must reproduce bit for bit) and "f64" (same sequence in binary64, the
reference for fitted parameters).
"""
import ctypes
import dataclasses
import os

import numpy as np

from . import build as _build

VALID, STOP_SINPHI, STOP_ARC, SPD_FAIL, REFIT64 = 1, 2, 4, 8, 16

_lib = None


@dataclasses.dataclass
class Params:
    bz: float = 0.5
    sigma_y: float = 0.1
    sigma_z: float = 0.1
    nf_win_y: float = 3.0
    nf_win_z: float = 3.0
    nf_chi2_max: float = 0.2
    tc_gate_nsigma: float = 3.0
    tc_max_miss: int = 4
    min_hits: int = 10
    precision: int = 0


class _P(ctypes.Structure):
    _fields_ = [("bz", ctypes.c_float), ("sigma_y", ctypes.c_float), ("sigma_z", ctypes.c_float),
                ("nf_win_y", ctypes.c_float), ("nf_win_z", ctypes.c_float), ("nf_chi2_max", ctypes.c_float),
                ("tc_gate_nsigma", ctypes.c_float), ("tc_max_miss", ctypes.c_int32),
                ("min_hits", ctypes.c_int32), ("precision", ctypes.c_int32)]


def _cp(p: Params):
    return _P(*dataclasses.astuple(p))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        for sfx, real in (("_f32", ctypes.c_float), ("_f64", ctypes.c_double)):
            getattr(L, "oracle_neighbours" + sfx).argtypes = [i32, vp, i32, vp, vp, vp, vp, vp, vp]
            getattr(L, "oracle_tracklets" + sfx).argtypes = [i32, vp, i32, vp, vp, vp, vp, i32, vp, vp] + [vp] * 10
            getattr(L, "oracle_refit" + sfx).argtypes = [i32, vp, i32, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp]
            getattr(L, "oracle_init" + sfx).argtypes = [vp, vp, vp, vp]
            getattr(L, "oracle_propagate" + sfx).argtypes = [vp, real, vp]
            getattr(L, "oracle_update" + sfx).argtypes = [vp, real, real, vp]
            getattr(L, "oracle_spd" + sfx).argtypes = [vp]
        L.oracle_clean_links.argtypes = [i32, vp, vp, vp, vp, vp]
        L.oracle_select.argtypes = [i32, i32, i32, vp, vp, vp, i32, vp, vp, vp, vp]
        L.oracle_fullfit_f32.argtypes = [i32, vp, i32, vp, vp, vp, ctypes.c_float, vp, i32, vp, vp, vp, vp, vp, vp,
                                         vp]
        L.oracle_fullfit_f64.argtypes = [i32, vp, i32, vp, vp, vp, ctypes.c_double, vp, i32, vp, vp, vp, vp, vp,
                                         vp, vp]
        L.oracle_merge.argtypes = [i32, vp, vp, vp, i32] + [vp] * 11
        L.oracle_fullfit_transport_f32.argtypes = [vp, vp, vp, ctypes.c_float, vp]
        L.oracle_fullfit_transport_f64.argtypes = [vp, vp, vp, ctypes.c_double, vp]
        L.oracle_refit_mixed.argtypes = [i32, vp, i32, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp]
        for f in ("oracle_neighbours_f32", "oracle_neighbours_f64", "oracle_tracklets_f32",
                  "oracle_tracklets_f64", "oracle_refit_f32", "oracle_refit_f64", "oracle_clean_links",
                  "oracle_refit_mixed", "oracle_init_f32", "oracle_init_f64", "oracle_propagate_f32",
                  "oracle_propagate_f64", "oracle_update_f32", "oracle_update_f64", "oracle_spd_f32",
                  "oracle_spd_f64", "oracle_select", "oracle_fullfit_f32", "oracle_fullfit_f64",
                  "oracle_fullfit_transport_f32", "oracle_fullfit_transport_f64", "oracle_merge"):
            getattr(L, f).restype = i32
        _lib = L
    return _lib


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _real(mode):
    if mode not in ("f32", "f64"):
        raise ValueError(mode)
    return np.float32 if mode == "f32" else np.float64


def neighbours(y, z, row, row_x, params=Params(), mode="f32"):
    """Neighbour finding: returns (link_up, link_dn), sector-local indices or -1."""
    y, z, row, rx = _c(y, np.float32), _c(z, np.float32), _c(row, np.int32), _c(row_x, np.float32)
    n = len(y)
    up = np.empty(n, np.int32)
    dn = np.empty(n, np.int32)
    p = _cp(params)
    rc = getattr(lib(), "oracle_neighbours_" + mode)(len(rx), rx.ctypes.data, n, y.ctypes.data, z.ctypes.data,
                                                      row.ctypes.data, ctypes.addressof(p), up.ctypes.data,
                                                      dn.ctypes.data)
    if rc:
        raise ValueError("hits are not row-sorted or a row is out of range")
    return up, dn


def clean_links(up, dn):
    """Mutual-link cleaning and start hits: (up_clean, dn_clean, start list)."""
    up, dn = _c(up, np.int32), _c(dn, np.int32)
    n = len(up)
    uc = np.empty(n, np.int32)
    dc = np.empty(n, np.int32)
    st = np.empty(n, np.uint8)
    lib().oracle_clean_links(n, up.ctypes.data, dn.ctypes.data, uc.ctypes.data, dc.ctypes.data, st.ctypes.data)
    return uc, dc, np.flatnonzero(st).astype(np.int32)


def select(n_hits, row_hit, n_hits_trk, flags, min_hits=10):
    """Tracklet selection of one sector (oracle/select.c).  Returns
    (owned [n_trk], tracks: list of (tracklet index, kept hits by row))."""
    rh = _c(row_hit, np.int32)
    n_trk = rh.shape[0] if rh.ndim == 2 else 0
    n_rows = rh.shape[1] if rh.ndim == 2 else 0
    nt_ = _c(n_hits_trk, np.int32)
    fl = _c(flags, np.int32)
    owned = np.zeros(max(n_trk, 1), np.int32)
    hits = np.zeros(max(int(n_trk) * max(n_rows, 1), 1), np.int32)
    cnt = np.zeros(2, np.int32)
    rc = lib().oracle_select(int(n_hits), n_rows, n_trk, rh.ctypes.data, nt_.ctypes.data, fl.ctypes.data,
                             int(min_hits), owned.ctypes.data, hits.ctypes.data, cnt[0:].ctypes.data,
                             cnt[1:].ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle_select failed ({rc})")
    owned = owned[:n_trk]
    tracks, pos = [], 0
    for t in np.flatnonzero(owned):
        k = int(owned[t])
        tracks.append((int(t), hits[pos:pos + k].copy()))
        pos += k
    assert len(tracks) == cnt[0] and pos == cnt[1]
    return owned, tracks


def fullfit(row_x, rows, hy, hz, x_start, p_start, start_row, p=None, mode="f64"):
    """Full Kalman refit of one track (oracle/fullfit.c): hits by ascending
    row, start state at row start_row.  Returns dict x, param[5], cov[15]
    (packed lower triangle over y, z, sin phi, tan lambda, q/pT), chi2, ndf,
    flags, at the outermost hit."""
    p = p or Params()
    real = np.float32 if mode == "f32" else np.float64
    rx = _c(row_x, np.float32)
    rows, hy, hz = _c(rows, np.int32), _c(hy, np.float32), _c(hz, np.float32)
    ps = _c(p_start, real)
    x = np.zeros(1, real)
    par = np.zeros(5, real)
    cov = np.zeros(15, real)
    chi2 = np.zeros(1, real)
    ndf = np.zeros(1, np.int32)
    fl = np.zeros(1, np.int32)
    cp = _cp(p)
    fn = lib().oracle_fullfit_f32 if mode == "f32" else lib().oracle_fullfit_f64
    fn(len(rx), rx.ctypes.data, len(rows), rows.ctypes.data, hy.ctypes.data, hz.ctypes.data, real(x_start),
       ps.ctypes.data, int(start_row), ctypes.byref(cp), x.ctypes.data, par.ctypes.data, cov.ctypes.data,
       chi2.ctypes.data, ndf.ctypes.data, fl.ctypes.data)
    return {"x": x[0], "param": par, "cov": cov, "chi2": chi2[0], "ndf": int(ndf[0]), "flags": int(fl[0])}


class _MP(ctypes.Structure):
    _fields_ = [("max_gap", ctypes.c_int32), ("window", ctypes.c_float), ("chi2_max", ctypes.c_float)]


@dataclasses.dataclass
class MergeParams:
    max_gap: int = 30
    window: float = 10.0
    chi2_max: float = 25.0


def merge(row_x, ok, a_last, e_x, e_p, e_C, b_first, s_x, s_p, s_C, p=None, mp=None):
    """Segment merging of one sector (oracle/merge.c): returns (next, chi2)."""
    p = p or Params()
    mp = mp or MergeParams()
    n = len(ok)
    rx = _c(row_x, np.float32)
    arrs = [_c(ok, np.int32), _c(a_last, np.int32), _c(e_x, np.float32), _c(e_p, np.float32).reshape(-1),
            _c(e_C, np.float32).reshape(-1), _c(b_first, np.int32), _c(s_x, np.float32),
            _c(s_p, np.float32).reshape(-1), _c(s_C, np.float32).reshape(-1)]
    for a, m in zip(arrs, (1, 1, 1, 5, 15, 1, 1, 5, 15)):
        assert a.size == n * m
    nxt = np.full(max(n, 1), -1, np.int32)
    chi2 = np.full(max(n, 1), -1.0, np.float32)
    lib().oracle_merge(len(rx), rx.ctypes.data, ctypes.byref(_cp(p)),
                       ctypes.byref(_MP(int(mp.max_gap), float(mp.window), float(mp.chi2_max))), n,
                       *[a.ctypes.data for a in arrs], nxt.ctypes.data, chi2.ctypes.data)
    return nxt[:n], chi2[:n]


def fullfit_transport(x, param, cov, x1, p=None, mode="f64"):
    """One transport step of the refit: returns (x, param, cov, rc)."""
    p = p or Params()
    real = np.float32 if mode == "f32" else np.float64
    xx = np.array([x], real)
    pp = np.array(param, real)
    cc = np.array(cov, real)
    fn = lib().oracle_fullfit_transport_f32 if mode == "f32" else lib().oracle_fullfit_transport_f64
    rc = fn(xx.ctypes.data, pp.ctypes.data, cc.ctypes.data, real(x1), ctypes.byref(_cp(p)))
    return xx[0], pp, cc, rc


def _trk_out(m, n_rows, real):
    return {"x_ref": np.empty(m, real), "param": np.empty((m, 5), real), "cov": np.empty((m, 15), real),
            "row_hit": np.empty((m, n_rows), np.int32), "start_row": np.empty(m, np.int32),
            "first_row": np.empty(m, np.int32), "last_row": np.empty(m, np.int32),
            "n_hits": np.empty(m, np.int32), "flags": np.empty(m, np.int32)}


def tracklets(y, z, row, row_x, up_clean, start, params=Params(), mode="f32"):
    """Tracklet construction for the given start hits; dict of per-tracklet arrays
    plus 'counters' = [transports, updates, gated candidates, row searches]."""
    y, z, row, rx = _c(y, np.float32), _c(z, np.float32), _c(row, np.int32), _c(row_x, np.float32)
    uc, st = _c(up_clean, np.int32), _c(start, np.int32)
    real = _real(mode)
    m = len(st)
    o = _trk_out(m, len(rx), real)
    cnt = np.zeros(4, np.int64)
    p = _cp(params)
    rc = getattr(lib(), "oracle_tracklets_" + mode)(
        len(rx), rx.ctypes.data, len(y), y.ctypes.data, z.ctypes.data, row.ctypes.data, uc.ctypes.data, m,
        st.ctypes.data, ctypes.addressof(p), o["x_ref"].ctypes.data, o["param"].ctypes.data,
        o["cov"].ctypes.data, o["row_hit"].ctypes.data, o["start_row"].ctypes.data, o["first_row"].ctypes.data,
        o["last_row"].ctypes.data, o["n_hits"].ctypes.data, o["flags"].ctypes.data, cnt.ctypes.data)
    if rc:
        raise ValueError("hits are not row-sorted or a row is out of range")
    o["counters"] = cnt
    return o


def refit(y, z, row_x, row_hit, start_row, params=Params(), mode="f64"):
    """Refit on recorded hit lists (no search).  Returns x_ref, param, cov, flags
    (flags bit 0: the refit reached the innermost hit)."""
    y, z, rx = _c(y, np.float32), _c(z, np.float32), _c(row_x, np.float32)
    rh, sr = _c(row_hit, np.int32), _c(start_row, np.int32)
    real = _real(mode)
    m = len(sr)
    x_ref, param, cov = np.empty(m, real), np.empty((m, 5), real), np.empty((m, 15), real)
    fl = np.empty(m, np.int32)
    p = _cp(params)
    getattr(lib(), "oracle_refit_" + mode)(len(rx), rx.ctypes.data, len(y), y.ctypes.data, z.ctypes.data, m,
                                           rh.ctypes.data, sr.ctypes.data, ctypes.addressof(p),
                                           x_ref.ctypes.data, param.ctypes.data, cov.ctypes.data, fl.ctypes.data)
    return {"x_ref": x_ref, "param": param, "cov": cov, "flags": fl}


def refit_mixed(y, z, row_x, row_hit, start_row, params=Params()):
    """Precision-form refit (binary32 state, binary64 covariance)."""
    y, z, rx = _c(y, np.float32), _c(z, np.float32), _c(row_x, np.float32)
    rh, sr = _c(row_hit, np.int32), _c(start_row, np.int32)
    m = len(sr)
    x_ref, param, cov = np.empty(m, np.float32), np.empty((m, 5), np.float32), np.empty((m, 15), np.float32)
    ok = np.empty(m, np.int32)
    p = _cp(params)
    lib().oracle_refit_mixed(len(rx), rx.ctypes.data, len(y), y.ctypes.data, z.ctypes.data, m, rh.ctypes.data,
                             sr.ctypes.data, ctypes.addressof(p), x_ref.ctypes.data, param.ctypes.data,
                             cov.ctypes.data, ok.ctypes.data)
    return {"x_ref": x_ref, "param": param, "cov": cov, "spd_ok": ok}


# state vector: x, y, z, s, l, q, c_yy, c_sy, c_ss, c_qy, c_qs, c_qq, c_zz, c_lz, c_ll
def init_state(h0, h1, params=Params(), mode="f64"):
    real = _real(mode)
    a, b = _c(h0, real), _c(h1, real)
    st = np.empty(15, real)
    p = _cp(params)
    rc = getattr(lib(), "oracle_init_" + mode)(a.ctypes.data, b.ctypes.data, ctypes.addressof(p), st.ctypes.data)
    return st, rc


def propagate(state, x1, params=Params(), mode="f64"):
    real = _real(mode)
    st = np.array(state, dtype=real)
    p = _cp(params)
    rc = getattr(lib(), "oracle_propagate_" + mode)(st.ctypes.data, real(x1), ctypes.addressof(p))
    return st, rc


def update(state, my, mz, params=Params(), mode="f64"):
    real = _real(mode)
    st = np.array(state, dtype=real)
    p = _cp(params)
    rc = getattr(lib(), "oracle_update_" + mode)(st.ctypes.data, real(my), real(mz), ctypes.addressof(p))
    return st, rc


def spd(state, mode="f64"):
    real = _real(mode)
    st = np.array(state, dtype=real)
    return bool(getattr(lib(), "oracle_spd_" + mode)(st.ctypes.data))


def track_sector(y, z, row, row_x, params=Params(), mode="f32"):
    """The whole hot path on one sector: neighbours, cleaning, start hits,
    tracklets.  Returns a dict with link_up/link_dn (raw), up_clean/dn_clean,
    start, and the tracklet arrays."""
    up, dn = neighbours(y, z, row, row_x, params, mode)
    uc, dc, start = clean_links(up, dn)
    out = tracklets(y, z, row, row_x, uc, start, params, mode)
    out.update({"link_up": up, "link_dn": dn, "up_clean": uc, "dn_clean": dc, "start": start})
    return out
