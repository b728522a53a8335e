"""Torch-facing wrapper of the catpc C ABI: device memory and streams only.

Torch supplies device buffers and the HIP stream; every computation runs in
libcatpc.so.  Nothing here computes tracking results.
"""
import ctypes

import numpy as np
import torch

from . import catpc as C


def _need_gpu(device):
    if not torch.cuda.is_available():
        raise RuntimeError("catpc needs a ROCm GPU (torch.cuda is not available)")
    return torch.device(device)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else ctypes.c_void_p(None)


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class DeviceHits:
    """Row-sorted hits of one or more sectors, resident on the device."""

    def __init__(self, y, z, row, hit_offset, device="cuda:0", x=None):
        dev = _need_gpu(device)
        self.device = dev
        self.hit_offset_host = np.ascontiguousarray(hit_offset, np.int64)
        self.y = torch.as_tensor(np.ascontiguousarray(y, np.float32)).to(dev)
        self.z = torch.as_tensor(np.ascontiguousarray(z, np.float32)).to(dev)
        self.row = torch.as_tensor(np.ascontiguousarray(row, np.int32)).to(dev)
        self.hit_offset = torch.as_tensor(self.hit_offset_host).to(dev)
        self.n_sectors = len(self.hit_offset_host) - 1
        self.n_hits = int(self.hit_offset_host[-1])
        s = C.catpc_input()
        s.y, s.z, s.row = _ptr(self.y), _ptr(self.z), _ptr(self.row)
        s.hit_offset = _ptr(self.hit_offset)
        s.hit_offset_host = ctypes.c_void_p(self.hit_offset_host.ctypes.data)
        s.n_sectors, s.n_hits = self.n_sectors, self.n_hits
        self.x = None if x is None else torch.as_tensor(np.ascontiguousarray(x, np.float32)).to(dev)
        s.x = _ptr(self.x)
        self.struct = s


class DeviceOutput:
    """Output buffers for n_hits hits, n_sectors sectors and `capacity` tracklets."""

    def __init__(self, n_hits, n_sectors, capacity, n_rows, device="cuda:0", keep_nf_links=True):
        dev = _need_gpu(device)
        e = lambda shape, dt: torch.empty(shape, dtype=dt, device=dev)
        i32 = torch.int32
        self.capacity = int(capacity)
        self.n_rows = n_rows
        self.link_up, self.link_dn = e(n_hits, i32), e(n_hits, i32)
        self.nf_up = e(n_hits, i32) if keep_nf_links else None
        self.nf_dn = e(n_hits, i32) if keep_nf_links else None
        self.start_hit = e(n_hits, i32)
        self.tracklet_offset = e(n_sectors + 1, torch.int64)
        cap = self.capacity
        self.x_ref = e(cap, torch.float32)
        self.param = e((cap, 5), torch.float32)
        self.cov = e((cap, 15), torch.float32)
        self.row_stride = C.catpc_row_stride(n_rows)
        self.row_hit = e((cap, self.row_stride), i32)  # [slot][row stride]
        self.start_row, self.first_row, self.last_row = e(cap, i32), e(cap, i32), e(cap, i32)
        self.n_hits, self.flags = e(cap, i32), e(cap, i32)
        s = C.catpc_output()
        for f in ("link_up", "link_dn", "nf_up", "nf_dn", "start_hit", "tracklet_offset", "x_ref", "param", "cov",
                  "row_hit", "start_row", "first_row", "last_row", "n_hits", "flags"):
            setattr(s, f, _ptr(getattr(self, f)))
        s.tracklet_capacity = cap
        self.struct = s

    def tracklets_numpy(self, n):
        n = min(int(n), self.capacity)
        g = lambda t: t[:n].cpu().numpy()
        return {"x_ref": g(self.x_ref), "param": g(self.param), "cov": g(self.cov),
                "row_hit": np.ascontiguousarray(self.row_hit[:n, :self.n_rows].cpu().numpy()),
                "start_row": g(self.start_row), "first_row": g(self.first_row), "last_row": g(self.last_row),
                "n_hits": g(self.n_hits), "flags": g(self.flags)}

    def links_numpy(self):
        d = {"link_up": self.link_up.cpu().numpy(), "link_dn": self.link_dn.cpu().numpy(),
             "tracklet_offset": self.tracklet_offset.cpu().numpy()}
        if self.nf_up is not None:
            d["nf_up"] = self.nf_up.cpu().numpy()
            d["nf_dn"] = self.nf_dn.cpu().numpy()
        off = d["tracklet_offset"]
        d["start_hit"] = self.start_hit[:int(off[-1])].cpu().numpy()
        return d


class DeviceTracks:
    """Output buffers of the tracklet selection: at most `track_capacity`
    tracks and `hit_capacity` track hits (n_hits always suffices)."""

    def __init__(self, n_sectors, track_capacity, hit_capacity, device="cuda:0"):
        dev = _need_gpu(device)
        e = lambda n, dt: torch.empty(n, dtype=dt, device=dev)
        self.track_offset = e(n_sectors + 1, torch.int64)
        self.track_tracklet = e(track_capacity, torch.int32)
        self.track_n_hits = e(track_capacity, torch.int32)
        self.track_hit_offset = e(track_capacity, torch.int64)
        self.track_hits = e(hit_capacity, torch.int32)
        s = C.catpc_tracks()
        for f in ("track_offset", "track_tracklet", "track_n_hits", "track_hit_offset", "track_hits"):
            setattr(s, f, _ptr(getattr(self, f)))
        s.track_capacity, s.hit_capacity = int(track_capacity), int(hit_capacity)
        self.struct = s

    def numpy(self, n_tracks, n_track_hits):
        return {"track_offset": self.track_offset.cpu().numpy(),
                "track_tracklet": self.track_tracklet[:n_tracks].cpu().numpy(),
                "track_n_hits": self.track_n_hits[:n_tracks].cpu().numpy(),
                "track_hit_offset": self.track_hit_offset[:n_tracks].cpu().numpy(),
                "track_hits": self.track_hits[:n_track_hits].cpu().numpy()}


class DeviceFits:
    """Output buffers of the full refit: one entry per track slot."""

    def __init__(self, capacity, device="cuda:0"):
        dev = _need_gpu(device)
        e = lambda shape, dt: torch.empty(shape, dtype=dt, device=dev)
        self.capacity = int(capacity)
        self.x = e(capacity, torch.float32)
        self.param = e((capacity, 5), torch.float32)
        self.cov = e((capacity, 15), torch.float32)
        self.chi2 = e(capacity, torch.float32)
        self.ndf = e(capacity, torch.int32)
        self.flags = e(capacity, torch.int32)
        s = C.catpc_fits()
        for f in ("x", "param", "cov", "chi2", "ndf", "flags"):
            setattr(s, f, _ptr(getattr(self, f)))
        s.capacity = self.capacity
        self.struct = s

    def numpy(self, n):
        g = lambda t: t[:n].cpu().numpy()
        return {"x": g(self.x), "param": g(self.param), "cov": g(self.cov), "chi2": g(self.chi2),
                "ndf": g(self.ndf), "flags": g(self.flags)}


class DeviceMerges:
    """Output buffers of the segment merging: one entry per track slot."""

    def __init__(self, capacity, device="cuda:0"):
        dev = _need_gpu(device)
        e = lambda dt: torch.empty(capacity, dtype=dt, device=dev)
        self.capacity = int(capacity)
        self.next, self.prev, self.head = e(torch.int32), e(torch.int32), e(torch.int32)
        self.chi2 = e(torch.float32)
        s = C.catpc_merges()
        for f in ("next", "prev", "head", "chi2"):
            setattr(s, f, _ptr(getattr(self, f)))
        s.capacity = self.capacity
        self.struct = s

    def numpy(self, n):
        g = lambda t: t[:n].cpu().numpy()
        return {"next": g(self.next), "prev": g(self.prev), "head": g(self.head), "chi2": g(self.chi2)}


class Tracker:
    """One catpc context on one device."""

    def __init__(self, row_x, max_hits, max_sectors, params=None, tuning=None, device="cuda:0"):
        self.device = _need_gpu(device)
        self.row_x = np.ascontiguousarray(row_x, np.float32)
        self.n_rows = len(self.row_x)
        self.params = params if params is not None else C.catpc_default_params()
        with torch.cuda.device(self.device):
            self.ctx = C.catpc_create(self.row_x, self.params, max_hits, max_sectors)
        if tuning is not None:
            self.set_tuning(tuning)

    def close(self):
        if getattr(self, "ctx", None):
            C.catpc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        C.catpc_set_params(self.ctx, params)
        self.params = params

    def set_tuning(self, tuning):
        if isinstance(tuning, dict):
            t = C.catpc_get_tuning(self.ctx)
            for k, v in tuning.items():
                setattr(t, k, v)
            tuning = t
        C.catpc_set_tuning(self.ctx, tuning)

    def tuning(self):
        return C.catpc_get_tuning(self.ctx)

    def output(self, hits, capacity=None, keep_nf_links=True):
        cap = hits.n_hits // 3 + 1 if capacity is None else capacity
        return DeviceOutput(hits.n_hits, hits.n_sectors, cap, self.n_rows, self.device, keep_nf_links)

    def track(self, hits, out, form="batch"):
        """Enqueue the hot path on the current stream (asynchronous)."""
        with torch.cuda.device(self.device):
            fn = C.catpc_track_batch if form == "batch" else C.catpc_track_plain
            fn(self.ctx, hits.struct, out.struct, _stream(self.device))

    def result(self):
        """Synchronise; (status, n_tracklets)."""
        with torch.cuda.device(self.device):
            return C.catpc_result(self.ctx, _stream(self.device))

    def stage_times(self, hits, out):
        """Per-stage milliseconds of one batched run (HIP events on the stream)."""
        with torch.cuda.device(self.device):
            return C.catpc_stage_times(self.ctx, hits.struct, out.struct, _stream(self.device))

    def work_counts(self):
        with torch.cuda.device(self.device):
            return C.catpc_work_counts(self.ctx, _stream(self.device))

    def tracks_output(self, hits, out):
        """Selection buffers that always suffice for this output."""
        return DeviceTracks(hits.n_sectors, out.capacity, max(hits.n_hits, 1), self.device)

    def select(self, hits, out, tracks):
        """Enqueue the tracklet selection of the last track call's output."""
        with torch.cuda.device(self.device):
            C.catpc_select_tracklets(self.ctx, hits.struct, out.struct, tracks.struct, _stream(self.device))

    def fits_output(self, tracks):
        """Refit buffers for every track slot of `tracks`."""
        return DeviceFits(max(int(tracks.struct.track_capacity), 1), self.device)

    def refit(self, hits, out, tracks, fits):
        """Enqueue the full Kalman refit of the selected tracks."""
        with torch.cuda.device(self.device):
            C.catpc_refit_tracks(self.ctx, hits.struct, out.struct, tracks.struct, fits.struct, _stream(self.device))

    def merges_output(self, tracks):
        """Merge buffers for every track slot of `tracks`."""
        return DeviceMerges(max(int(tracks.struct.track_capacity), 1), self.device)

    def merge(self, hits, out, tracks, fits, merges, cuts=None):
        """Enqueue the merging of track segments inside each sector; `cuts`
        (catpc_merge_params) None takes the defaults."""
        with torch.cuda.device(self.device):
            C.catpc_merge_tracks(self.ctx, hits.struct, out.struct, tracks.struct, fits.struct, cuts,
                                 merges.struct, _stream(self.device))

    def merge_counts(self):
        """Synchronise; (candidate pairs, transport row steps) of the last merge."""
        with torch.cuda.device(self.device):
            return C.catpc_merge_counts(self.ctx, _stream(self.device))

    def select_result(self):
        """Synchronise; (n_tracks, n_track_hits)."""
        with torch.cuda.device(self.device):
            return C.catpc_select_result(self.ctx, _stream(self.device))

    def fetch(self, hits, first, out):
        with torch.cuda.device(self.device):
            C.catpc_fetch_tracklets(self.ctx, hits.struct, first, out.struct, _stream(self.device))
