"""Serving form: a stream of events tracked with continuous batching.

Events arrive over time (e.g. Poisson, Sec. 1: ALICE records heavy-ion
collisions at up to ~1 kHz).  The server keeps several in-flight slots, each
a catpc context with its own HIP stream, device-resident workspace (the row
grids never leave the device) and device input/output buffers.  Whenever a
slot is free, every event that has arrived and is still waiting (FIFO, as far
as the slot's capacity allows) is admitted into one batch: its hits go up in
one host-to-device copy from pinned memory, the batched chain runs on the
slot's stream, and an estimated share of the tracklet output comes back in
one device-to-host copy queued right behind it; tracklets beyond the estimate
are fetched afterwards (Sec. 3.1: estimate the output buffer, fetch the rest
later).  Batches on different slots overlap on the device (Sec. 3.2: several
independent tracker instances on one GPU).

Admission is bounded by an HBM budget (Sec. 3.2: further events go onto the
GPU as long as its memory suffices).  Every in-flight batch is charged its
footprint by the paper's memory model (Sec. 4.1: the tracker's internal
memory is about three times its input): input + 3 x input + outputs (links,
start list, and the estimated tracklet records), from the batch's own hit
and sector counts.  A free slot takes the waiting events (FIFO) only as far
as the in-flight footprint stays within the budget; an arrived event that
does not fit waits for a completion (a budget deferral), even with a slot
free.  The number of slots is how many batches of the stream's largest event
fit in the budget, at most `n_slots`; each slot's buffers are allocated once,
for its capacity (`slot_hits`, `slot_sectors`).

Latency of an event = completion of its batch (results in host memory)
minus its arrival time.  Nothing here computes tracking results: every step
runs in libcatpc.so.
"""
import ctypes
import time

import numpy as np
import torch

from . import catpc as C
from .tracker import Tracker, _ptr

TRACKLET_FIELDS = (("x_ref", np.float32, ()), ("param", np.float32, (5,)), ("cov", np.float32, (15,)),
                   ("start_row", np.int32, ()), ("first_row", np.int32, ()), ("last_row", np.int32, ()),
                   ("n_hits", np.int32, ()), ("flags", np.int32, ()))
BYTES_PER_TRACKLET = 4 * (1 + 5 + 15 + 5)  # plus 4 * row stride for the hit-per-row record


class EventStream:
    """A stream of events drawn from a pool held in pinned host memory.

    pool: synth.Batch-like objects (one event each: y, z, row, hit_offset over
    its sectors), stored once, concatenated, in pinned memory (the events'
    host buffers).  order: pool index of each arriving event.  arrival:
    arrival time of each event (s, from stream start)."""

    def __init__(self, pool, order, arrival, row_x):
        self.row_x = np.asarray(row_x, np.float32)
        self.order = np.asarray(order, np.int64)
        self.arrival = np.asarray(arrival, np.float64)
        p_hits = np.array([ev.n_hits for ev in pool], np.int64)
        p_secs = np.array([ev.n_sectors for ev in pool], np.int64)
        self.pool_hit0 = np.concatenate([[0], np.cumsum(p_hits)])
        self.pool_off = [np.asarray(ev.hit_offset, np.int64) for ev in pool]
        H = int(self.pool_hit0[-1])
        pin = lambda n, dt: torch.empty(n, dtype=dt, pin_memory=True)
        self.y, self.z, self.row = pin(H, torch.float32), pin(H, torch.float32), pin(H, torch.int32)
        yn, zn, rn = self.y.numpy(), self.z.numpy(), self.row.numpy()
        for i, ev in enumerate(pool):
            a, b = int(self.pool_hit0[i]), int(self.pool_hit0[i + 1])
            yn[a:b], zn[a:b], rn[a:b] = ev.y, ev.z, ev.row
        self.n_events = len(self.order)
        self.ev_hits = p_hits[self.order]
        self.ev_secs = p_secs[self.order]
        # running totals over the stream (batch sizes are differences)
        self.hit_start = np.concatenate([[0], np.cumsum(self.ev_hits)])
        self.sec_start = np.concatenate([[0], np.cumsum(self.ev_secs)])


class Slot:
    """One in-flight batch: a catpc context, a stream, device buffers."""

    def __init__(self, row_x, max_hits, max_sectors, params, tuning, device, out_frac, keep_rows):
        self.device = torch.device(device)
        self.max_hits, self.max_sectors = int(max_hits), int(max_sectors)
        tun = dict(tuning or {})
        tun["use_graph"] = 0  # sizes change from batch to batch
        self.tracker = Tracker(row_x, self.max_hits, self.max_sectors, params=params, tuning=tun, device=device)
        self.n_rows = len(row_x)
        self.stream = torch.cuda.Stream(device=self.device)
        e = lambda n, dt: torch.empty(n, dtype=dt, device=self.device)
        self.y, self.z, self.row = e(max_hits, torch.float32), e(max_hits, torch.float32), e(max_hits, torch.int32)
        self.hit_offset = e(max_sectors + 1, torch.int64)
        self.off_host = torch.empty(max_sectors + 1, dtype=torch.int64, pin_memory=True)
        self.cap = self.max_hits // 3 + 1
        self.out = self.tracker.output(_Sizes(max_hits, max_sectors), self.cap, keep_nf_links=False)
        self.out_frac = out_frac
        self.est = max(4096, int(out_frac * max_hits))
        self.keep_rows = keep_rows
        pin = lambda shape, dt: torch.empty(shape, dtype=dt, pin_memory=True)
        self.h_toff = pin(max_sectors + 1, torch.int64)
        self.h_trk = {f: pin((self.est,) + sh, getattr(torch, np.dtype(dt).name)) for f, dt, sh in TRACKLET_FIELDS}
        self.h_rows = pin((self.est, self.out.row_stride), torch.int32) if keep_rows else None
        self.done = torch.cuda.Event()
        self.busy = False
        self.events = None
        self.late_fetches = 0
        self.inp = C.catpc_input()

    def reserved(self):
        """Device bytes the slot holds: workspace, input and output buffers."""
        ws = C.catpc_workspace_bytes(self.n_rows, self.max_hits, self.max_sectors)
        inputs = 12 * self.max_hits + 8 * (self.max_sectors + 1)
        outputs = 12 * self.max_hits + 8 * (self.max_sectors + 1) + self.cap * (BYTES_PER_TRACKLET + 4 * self.out.row_stride)
        return ws + inputs + outputs

    def charge(self, n_hits, n_sectors):
        """Footprint of a batch of n_hits hits in n_sectors sectors."""
        est = min(self.est, max(256, int(self.out_frac * n_hits)))
        return batch_footprint(n_hits, n_sectors, est, self.out.row_stride)

    def submit(self, stream_src, e0, e1):
        """Enqueue events [e0, e1) of the stream: H2D of each event's hits into
        the batch buffer, the hot path, D2H of an estimated share of the
        output."""
        S = stream_src
        n = int(S.hit_start[e1] - S.hit_start[e0])
        ns = int(S.sec_start[e1] - S.sec_start[e0])
        off = self.off_host.numpy()
        with torch.cuda.stream(self.stream):
            h, sec = 0, 0
            for e in range(e0, e1):
                p = int(S.order[e])
                a, m = int(S.pool_hit0[p]), int(S.ev_hits[e])
                self.y[h:h + m].copy_(S.y[a:a + m], non_blocking=True)
                self.z[h:h + m].copy_(S.z[a:a + m], non_blocking=True)
                self.row[h:h + m].copy_(S.row[a:a + m], non_blocking=True)
                po = S.pool_off[p]
                off[sec:sec + len(po)] = h + po
                h += m
                sec += len(po) - 1
            self.hit_offset[:ns + 1].copy_(self.off_host[:ns + 1], non_blocking=True)
            inp = self.inp
            inp.y, inp.z, inp.row = _ptr(self.y), _ptr(self.z), _ptr(self.row)
            inp.hit_offset = _ptr(self.hit_offset)
            inp.hit_offset_host = ctypes.c_void_p(None)
            inp.n_sectors, inp.n_hits = ns, n
            C.catpc_track_batch(self.tracker.ctx, inp, self.out.struct,
                                ctypes.c_void_p(self.stream.cuda_stream))
            est = min(self.est, max(256, int(self.out_frac * n)))
            self.h_toff[:ns + 1].copy_(self.out.tracklet_offset[:ns + 1], non_blocking=True)
            for f, _, _ in TRACKLET_FIELDS:
                self.h_trk[f][:est].copy_(getattr(self.out, f)[:est], non_blocking=True)
            if self.keep_rows:
                self.h_rows[:est].copy_(self.out.row_hit[:est], non_blocking=True)
            self.done.record(self.stream)
        self.busy = True
        self.events = (e0, e1, ns, est)
        self.charged = self.charge(n, ns)

    def collect(self, keep):
        """After the batch completed: status check, late fetch of tracklets
        beyond the estimate, per-event results (if keep)."""
        with torch.cuda.stream(self.stream):
            st, n_trk = self.tracker.result()
        if st != C.CATPC_OK:
            raise C.CatpcError(st, C.catpc_last_error())
        e0, e1, ns, est = self.events
        trk = {f: self.h_trk[f].numpy()[:min(n_trk, est)] for f, _, _ in TRACKLET_FIELDS}
        rows = self.h_rows.numpy()[:min(n_trk, est), :self.n_rows] if self.keep_rows else None
        self.late_fetches += int(n_trk > est)
        if n_trk > est:  # late fetch of the remainder
            with torch.cuda.stream(self.stream):
                extra = {f: getattr(self.out, f)[est:n_trk].cpu().numpy() for f, _, _ in TRACKLET_FIELDS}
                if self.keep_rows:
                    rows = np.concatenate([rows, self.out.row_hit[est:n_trk, :self.n_rows].cpu().numpy()])
            trk = {f: np.concatenate([trk[f], extra[f]]) for f in trk}
        self.busy = False
        res = None
        if keep:
            toff = self.h_toff.numpy()[:ns + 1].copy()
            res = {"toff": toff, "trk": {f: v.copy() for f, v in trk.items()},
                   "rows": None if rows is None else rows.copy()}
        return n_trk, res


def batch_footprint(n_hits, n_sectors, est_tracklets, row_stride):
    """HBM charged to a batch: input (y, z, row, sector offsets) + three
    times the input for the tracker's internal memory + outputs (links and
    start list, per-sector tracklet offsets, the estimated tracklet records)."""
    inp = 12 * n_hits + 8 * (n_sectors + 1)
    out = 12 * n_hits + 8 * (n_sectors + 1) + est_tracklets * (BYTES_PER_TRACKLET + 4 * row_stride)
    return inp + 3 * inp + out


class _Sizes:
    def __init__(self, n_hits, n_sectors):
        self.n_hits, self.n_sectors = n_hits, n_sectors


def serve(stream_src, n_slots=3, slot_hits=4_000_000, slot_sectors=36 * 24, hbm_budget=64 << 30,
          params=None, tuning=None, device="cuda:0", out_frac=0.03, keep_results=False, keep_rows=False,
          warmup_events=0, realtime=True):
    """Run the event stream; returns a dict with per-event latency (s), batch
    sizes, sustained hits/s, the in-flight footprint and budget deferrals, and
    (optionally) per-event results."""
    S = stream_src
    if int(S.ev_hits.max(initial=0)) > slot_hits or int(S.ev_secs.max(initial=0)) > slot_sectors:
        raise ValueError("an event exceeds the slot capacity")
    first = Slot(S.row_x, slot_hits, slot_sectors, params, tuning, device, out_frac, keep_rows)
    full = first.charge(slot_hits, slot_sectors)
    biggest = max(first.charge(int(h), int(k)) for h, k in zip(S.ev_hits, S.ev_secs)) if S.n_events else 1
    if biggest > hbm_budget:
        first.tracker.close()
        raise ValueError("an event's footprint exceeds the HBM budget")
    # as many slots as batches of the largest event fit in the budget, at most n_slots
    want = max(1, min(n_slots, hbm_budget // biggest))
    slots = [first] + [Slot(S.row_x, slot_hits, slot_sectors, params, tuning, device, out_frac, keep_rows)
                       for _ in range(want - 1)]
    torch.cuda.synchronize(device)
    n = S.n_events
    done_t = np.zeros(n)
    batch_of = np.full(n, -1, np.int64)
    results = [None] * n if keep_results else None
    batches = []
    nxt = 0          # next event not yet admitted
    finished = 0
    in_flight = 0    # footprint charged to the batches on the device
    peak = 0
    deferred = set()  # events that waited with a slot free because the budget was spent
    t0 = time.perf_counter()
    while finished < n:
        now = time.perf_counter() - t0
        # completions
        for sl in slots:
            if sl.busy and sl.done.query():
                e0, e1 = sl.events[0], sl.events[1]
                n_trk, res = sl.collect(keep_results)
                in_flight -= sl.charged
                tdone = time.perf_counter() - t0
                done_t[e0:e1] = tdone
                finished += e1 - e0
                if keep_results:
                    split_events(S, e0, e1, res, results)
        # admissions: arrived events go into free slots as whole FIFO batches, within the budget
        if not realtime:
            now = float("inf")
        for sl in slots:
            if sl.busy or nxt >= n or S.arrival[nxt] > now:
                continue
            e1 = nxt
            while (e1 < n and S.arrival[e1] <= now and
                   S.hit_start[e1 + 1] - S.hit_start[nxt] <= sl.max_hits and
                   S.sec_start[e1 + 1] - S.sec_start[nxt] <= sl.max_sectors and
                   in_flight + sl.charge(int(S.hit_start[e1 + 1] - S.hit_start[nxt]),
                                         int(S.sec_start[e1 + 1] - S.sec_start[nxt])) <= hbm_budget):
                e1 += 1
            if e1 == nxt:  # the next event does not fit in what is left of the budget
                deferred.add(nxt)
                break
            sl.submit(S, nxt, e1)
            in_flight += sl.charged
            peak = max(peak, in_flight)
            batch_of[nxt:e1] = len(batches)
            batches.append(e1 - nxt)
            nxt = e1
        if realtime and nxt < n and not any(sl.busy for sl in slots):
            wait = S.arrival[nxt] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.0005))
    lat = done_t - S.arrival
    w = slice(warmup_events, n)
    span = done_t[w].max() - S.arrival[w].min() if n > warmup_events else 0.0
    hits = float(S.ev_hits[w].sum())
    out = {"latency_s": lat, "p50_ms": float(np.percentile(lat[w], 50) * 1e3) if n > warmup_events else None,
           "p99_ms": float(np.percentile(lat[w], 99) * 1e3) if n > warmup_events else None,
           "hits_per_s": hits / span if span > 0 else None, "n_events": n - warmup_events,
           "batches": len(batches), "mean_batch_events": float(np.mean(batches)) if batches else 0.0,
           "batch_of": batch_of, "slots": len(slots), "slot_reserved_bytes": slots[0].reserved(),
           "full_batch_footprint_bytes": full, "hbm_budget_bytes": hbm_budget,
           "peak_in_flight_bytes": peak, "deferred_events": len(deferred),
           "largest_event_footprint_bytes": biggest,
           "late_fetches": sum(sl.late_fetches for sl in slots),
           "results": results}
    for sl in slots:
        sl.tracker.close()
    return out


def split_events(S, e0, e1, res, results):
    """Per-event slices of a batch's results (sector-local indices, so they
    are the same whatever batch the event was in)."""
    toff = res["toff"]
    s_base = int(S.sec_start[e0])
    for e in range(e0, e1):
        a, b = int(S.sec_start[e]) - s_base, int(S.sec_start[e + 1]) - s_base
        t0, t1 = int(toff[a]), int(toff[b])
        results[e] = {"toff": toff[a:b + 1] - toff[a],
                      "trk": {f: v[t0:t1] for f, v in res["trk"].items()},
                      "rows": None if res["rows"] is None else res["rows"][t0:t1]}


def poisson_arrivals(n, rate_hz, seed):
    """Arrival times (s) of a Poisson process: exponential gaps with mean
    1/rate, from a seeded generator."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_hz, n))
