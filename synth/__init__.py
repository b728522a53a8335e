"""Seeded synthetic TPC events (the detector simulation; no tracking arithmetic).

Every input the tests, the smoke check and the benchmark use comes from here:
primary helices from the origin in a constant field Bz, intersected with the
159 pad-row planes of the 36 sectors (Sec. 2: the TPC is split into two halves
of 18 trapezoidal sectors; Sec. 1: up to 159 hits per track), Gaussian smear,
and uniform noise hits.  The paper measures on recorded ALICE pp and Pb-Pb
events; these seeded events stand in for them with the same structure (one
hit per track and pad row, row-sorted per sector, sector multiplicities from
a few tens of tracks to a central heavy-ion event).

The generator is plain C (gen.c) driven through ctypes; it is compiled by
synth/build.py.
"""
import ctypes
import math
import os

import numpy as np

from . import build as _build

N_ROWS = 159
X_FIRST = 85.0
X_LAST = 247.0
TAN_HALF_OPEN = math.tan(math.radians(10.0))
Z_MAX = 250.0
BZ = 0.5
N_SECTORS = 36

_lib = None


class _Cfg(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int32),
                ("x_first", ctypes.c_double), ("x_last", ctypes.c_double),
                ("bz", ctypes.c_double), ("sigma", ctypes.c_double),
                ("noise_frac", ctypes.c_double), ("tan_half_open", ctypes.c_double),
                ("z_max", ctypes.c_double),
                ("pt_min", ctypes.c_double), ("pt_max", ctypes.c_double),
                ("eta_min", ctypes.c_double), ("eta_max", ctypes.c_double),
                ("phi_min", ctypes.c_double), ("phi_max", ctypes.c_double),
                ("sector_first", ctypes.c_int32), ("sector_count", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("dead_first", ctypes.c_int32), ("dead_count", ctypes.c_int32)]


_dp = ctypes.POINTER(ctypes.c_double)


class _Event(ctypes.Structure):
    _fields_ = [("n_sectors", ctypes.c_int32), ("n_hits", ctypes.c_int64),
                ("hit_offset", ctypes.POINTER(ctypes.c_int64)),
                ("x", ctypes.POINTER(ctypes.c_float)), ("y", ctypes.POINTER(ctypes.c_float)),
                ("z", ctypes.POINTER(ctypes.c_float)),
                ("row", ctypes.POINTER(ctypes.c_int32)), ("label", ctypes.POINTER(ctypes.c_int32)),
                ("y_true", _dp), ("z_true", _dp), ("sinphi_true", _dp),
                ("n_tracks", ctypes.c_int32),
                ("trk_q", _dp), ("trk_pt", _dp), ("trk_eta", _dp), ("trk_phi0", _dp)]


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        L.synth_generate.restype = ctypes.POINTER(_Event)
        L.synth_generate.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_int32, ctypes.c_uint32, ctypes.c_int32]
        L.synth_generate_tracks.restype = ctypes.POINTER(_Event)
        L.synth_generate_tracks.argtypes = [ctypes.POINTER(_Cfg), ctypes.c_int32] + [ctypes.c_void_p] * 4 + \
            [ctypes.c_uint32, ctypes.c_int32]
        L.synth_free.argtypes = [ctypes.POINTER(_Event)]
        L.synth_row_x.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_void_p]
        L.synth_sector_alpha.restype = ctypes.c_double
        L.synth_sector_alpha.argtypes = [ctypes.c_int32]
        L.synth_multiplicity.restype = ctypes.c_int32
        L.synth_multiplicity.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double, ctypes.c_double]
        L.synth_philox4x32_10.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.synth_helix_point.argtypes = [ctypes.c_double] * 6 + [ctypes.c_void_p]
        _lib = L
    return _lib


def row_x(n_rows=N_ROWS, x_first=X_FIRST, x_last=X_LAST):
    """Pad-row x positions (cm) as float32: evenly spaced, computed in double."""
    out = np.empty(n_rows, np.float32)
    lib().synth_row_x(n_rows, x_first, x_last, out.ctypes.data)
    return out


def sector_alpha(s):
    return lib().synth_sector_alpha(int(s))


def philox4x32_10(ctr, key):
    c = np.asarray(ctr, np.uint32)
    k = np.asarray(key, np.uint32)
    o = np.empty(4, np.uint32)
    lib().synth_philox4x32_10(c.ctypes.data, k.ctypes.data, o.ctypes.data)
    return o


def helix_point(q_over_pt, tanl, phi0, bz, alpha, path):
    """Closed-form helix from the origin in the sector frame rotated by alpha:
    returns (x, y, z, sin(phi_local)) at transverse path length `path`."""
    o = np.empty(4, np.float64)
    lib().synth_helix_point(q_over_pt, tanl, phi0, bz, alpha, path, o.ctypes.data)
    return o


def _cfg(seed, sectors, n_rows=N_ROWS, bz=BZ, sigma=0.1, noise_frac=0.1, pt=(0.2, 10.0),
         eta=(-0.9, 0.9), phi=(0.0, 2 * math.pi), dead_rows=(0, 0)):
    c = _Cfg()
    c.n_rows = n_rows
    c.x_first, c.x_last = X_FIRST, X_LAST
    c.bz, c.sigma, c.noise_frac = bz, sigma, noise_frac
    c.tan_half_open, c.z_max = TAN_HALF_OPEN, Z_MAX
    c.pt_min, c.pt_max = pt
    c.eta_min, c.eta_max = eta
    c.phi_min, c.phi_max = phi
    c.sector_first, c.sector_count = sectors
    c.seed = seed
    c.dead_first, c.dead_count = dead_rows
    return c


class Batch:
    """Concatenated sectors of one or more events, row-sorted per sector.

    x, y, z: float32[n]; row, label: int32[n]; hit_offset: int64[S+1];
    alpha: float64[S] (sector rotation, rad); side: int8[S] (+1 A, -1 C);
    sector_id, event_id: int32[S]; row_x: float32[159].  `truth` (optional)
    holds y_true, z_true, sinphi_true per hit and the track table per event.
    """

    def __init__(self, parts, n_rows=N_ROWS, bz=BZ):
        self.row_x = row_x(n_rows)
        self.bz = bz
        self.n_rows = n_rows
        xs, ys, zs, rows, labels = [], [], [], [], []
        offs = [0]
        sec_ids, ev_ids = [], []
        truth = {"y_true": [], "z_true": [], "sinphi_true": []}
        self.tracks = []
        has_truth = True
        for ev_id, sec_first, ev in parts:
            n = ev["n_hits"]
            base = offs[-1]
            for s in range(len(ev["hit_offset"]) - 1):
                offs.append(base + int(ev["hit_offset"][s + 1]))
                sec_ids.append(sec_first + s)
                ev_ids.append(ev_id)
            xs.append(ev["x"]); ys.append(ev["y"]); zs.append(ev["z"])
            rows.append(ev["row"]); labels.append(ev["label"])
            if ev.get("y_true") is None:
                has_truth = False
            else:
                for k in truth:
                    truth[k].append(ev[k])
            self.tracks.append(ev["tracks"])
            assert offs[-1] == base + n
        cat = lambda a, dt: np.ascontiguousarray(np.concatenate(a).astype(dt, copy=False)) if a else np.zeros(0, dt)
        self.x, self.y, self.z = cat(xs, np.float32), cat(ys, np.float32), cat(zs, np.float32)
        self.row, self.label = cat(rows, np.int32), cat(labels, np.int32)
        self.hit_offset = np.asarray(offs, np.int64)
        self.sector_id = np.asarray(sec_ids, np.int32)
        self.event_id = np.asarray(ev_ids, np.int32)
        self.alpha = np.array([sector_alpha(s) for s in self.sector_id], np.float64)
        self.side = np.where(self.sector_id < 18, 1, -1).astype(np.int8)
        self.truth = {k: cat(v, np.float64) for k, v in truth.items()} if has_truth else None

    @property
    def n_hits(self):
        return int(self.hit_offset[-1])

    @property
    def n_sectors(self):
        return len(self.hit_offset) - 1

    def sector(self, s):
        a, b = int(self.hit_offset[s]), int(self.hit_offset[s + 1])
        d = {"x": self.x[a:b], "y": self.y[a:b], "z": self.z[a:b], "row": self.row[a:b],
             "label": self.label[a:b], "alpha": float(self.alpha[s]), "sector_id": int(self.sector_id[s]),
             "event_id": int(self.event_id[s])}
        if self.truth is not None:
            for k, v in self.truth.items():
                d[k] = v[a:b]
        return d


def generate_event(seed, n_tracks, event_id=0, sectors=(0, N_SECTORS), truth=False, tracks=None, **kw):
    """One event as a dict of numpy arrays (sector-concatenated).  `tracks`
    (optional) = dict of arrays q (+-1), pt (GeV), eta, phi0 (rad) replacing the
    random track table; n_tracks is then its length."""
    c = _cfg(seed, sectors, **kw)
    L = lib()
    if tracks is None:
        p = L.synth_generate(ctypes.byref(c), int(n_tracks), int(event_id), 1 if truth else 0)
    else:
        arrs = [np.ascontiguousarray(tracks[k], np.float64) for k in ("q", "pt", "eta", "phi0")]
        n_tracks = len(arrs[0])
        p = L.synth_generate_tracks(ctypes.byref(c), n_tracks, *[a.ctypes.data for a in arrs], int(event_id),
                                    1 if truth else 0)
    if not p:
        raise MemoryError("synth_generate failed")
    try:
        e = p.contents
        n = int(e.n_hits)
        S = int(e.n_sectors)
        arr = lambda ptr, m, dt: np.ctypeslib.as_array(ptr, shape=(m,)).astype(dt, copy=True) if m > 0 else np.zeros(0, dt)
        out = {"n_hits": n,
               "hit_offset": arr(e.hit_offset, S + 1, np.int64),
               "x": arr(e.x, n, np.float32), "y": arr(e.y, n, np.float32), "z": arr(e.z, n, np.float32),
               "row": arr(e.row, n, np.int32), "label": arr(e.label, n, np.int32)}
        if truth:
            out["y_true"] = arr(e.y_true, n, np.float64)
            out["z_true"] = arr(e.z_true, n, np.float64)
            out["sinphi_true"] = arr(e.sinphi_true, n, np.float64)
        else:
            out["y_true"] = None
        T = int(e.n_tracks)
        out["tracks"] = {"q": arr(e.trk_q, T, np.float64), "pt": arr(e.trk_pt, T, np.float64),
                         "eta": arr(e.trk_eta, T, np.float64), "phi0": arr(e.trk_phi0, T, np.float64)}
    finally:
        L.synth_free(p)
    return out


# --------------------------------------------------------------- workloads
def sector_workload(seed=1, n_tracks=200, truth=False, **kw):
    """One A-side sector (s = 0): n_tracks primaries aimed at it (phi0 within
    +-10 deg of the sector axis, eta in [0, 0.9)), smear 0.1 cm, 10 % noise."""
    a0 = sector_alpha(0)
    kw.setdefault("eta", (0.0, 0.9))
    kw.setdefault("phi", (a0 - math.radians(10.0), a0 + math.radians(10.0)))
    ev = generate_event(seed, n_tracks, 0, sectors=(0, 1), truth=truth, **kw)
    return Batch([(0, 0, ev)], n_rows=kw.get("n_rows", N_ROWS), bz=kw.get("bz", BZ))


def tracks_workload(tracks, sector=0, seed=1, truth=True, **kw):
    """One sector from an explicit track table (see generate_event)."""
    ev = generate_event(seed, 0, 0, sectors=(sector, 1), truth=truth, tracks=tracks, **kw)
    return Batch([(0, sector, ev)], n_rows=kw.get("n_rows", N_ROWS), bz=kw.get("bz", BZ))


def event_workload(seed=1, n_tracks=10000, truth=False, **kw):
    """A full event: n_tracks primaries over all 36 sectors."""
    ev = generate_event(seed, n_tracks, 0, sectors=(0, N_SECTORS), truth=truth, **kw)
    return Batch([(0, 0, ev)], n_rows=kw.get("n_rows", N_ROWS), bz=kw.get("bz", BZ))


def multiplicities(seed, n_events, lo=20.0, hi=1.0e4):
    return [int(lib().synth_multiplicity(seed, e, lo, hi)) for e in range(n_events)]


def event_pool(seed=2, n_events=64, lo=20.0, hi=1.0e4, **kw):
    """n_events single-event Batches with the same multiplicity law as
    batch_workload (for streams of arriving events)."""
    mult = multiplicities(seed, n_events, lo, hi)
    from concurrent.futures import ThreadPoolExecutor
    work = lambda i: Batch([(i, 0, generate_event(seed, mult[i], i, sectors=(0, N_SECTORS), **kw))],
                           n_rows=kw.get("n_rows", N_ROWS), bz=kw.get("bz", BZ))
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        return list(ex.map(work, range(n_events)))


def batch_workload(seed=1, n_events=64, lo=20.0, hi=1.0e4, truth=False, first_event=0, **kw):
    """n_events events with multiplicity floor(exp(U(ln lo, ln hi))): 36 sectors
    each, from near-empty sectors to central-heavy-ion-like ones."""
    mult = multiplicities(seed, first_event + n_events, lo, hi)[first_event:]
    from concurrent.futures import ThreadPoolExecutor
    work = lambda i: generate_event(seed, mult[i], first_event + i, sectors=(0, N_SECTORS), truth=truth, **kw)
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        evs = list(ex.map(work, range(len(mult))))
    parts = [(first_event + i, 0, ev) for i, ev in enumerate(evs)]
    b = Batch(parts, n_rows=kw.get("n_rows", N_ROWS), bz=kw.get("bz", BZ))
    b.multiplicity = mult
    return b
