"""Scheduling baselines of the per-sector (plain) form, after Sec. 3.1 and
Sec. 3.2 of the paper: the same stage chains, only the way they are put on
the GPU differs.

- queues by sector (Sec. 3.1): the sectors of a batch are spread round-robin
  over Q command queues; each queue launches the chain sector by sector, and
  the GPU runs the queues concurrently;
- instances by event (Sec. 3.2): K independent tracker instances on one GPU,
  each taking whole events (round-robin) and launching them sector by sector
  (or, for comparison, as one batched chain).

Each queue or instance is a catpc context with its own workspace, stream and
device buffers (its share of the hits copied once, outside the timing).
Every sector's result is the same as in the single batched chain (all
indices are sector-local).  Nothing here computes tracking results.
"""
import numpy as np
import torch

from .tracker import DeviceHits, Tracker


class Queues:
    """Q contexts/streams over a synth.Batch-like object (y, z, row,
    hit_offset, event_id, row_x), split by "sector" or by "event"."""

    def __init__(self, batch, q, by="sector", form="plain", tuning=None, params=None, device="cuda:0"):
        if by not in ("sector", "event") or form not in ("plain", "batch") or q < 1:
            raise ValueError("by must be 'sector' or 'event', form 'plain' or 'batch', q >= 1")
        self.device = torch.device(device)
        self.form = form
        S = len(batch.hit_offset) - 1
        key = np.arange(S) if by == "sector" else np.asarray(batch.event_id)
        groups = np.unique(key)
        owner = {g: i % q for i, g in enumerate(groups)}
        self.sectors = [np.array([s for s in range(S) if owner[key[s]] == k], np.int64) for k in range(q)]
        self.parts = []
        for k in range(q):
            secs = self.sectors[k]
            if len(secs) == 0:
                continue
            a, b = batch.hit_offset[secs], batch.hit_offset[secs + 1]
            idx = np.concatenate([np.arange(x, y) for x, y in zip(a, b)]) if len(secs) else np.zeros(0, np.int64)
            off = np.concatenate([[0], np.cumsum(b - a)])
            hits = DeviceHits(batch.y[idx], batch.z[idx], batch.row[idx], off, device)
            tr = Tracker(batch.row_x, max(hits.n_hits, 1), max(hits.n_sectors, 1), params=params, device=device)
            tun = dict(tuning or {})
            if form == "plain":
                tun["use_graph"] = 0
            if tun:
                tr.set_tuning(tun)
            out = tr.output(hits)
            stream = torch.cuda.Stream(device=self.device)
            self.parts.append({"sectors": secs, "hits": hits, "tracker": tr, "out": out, "stream": stream})
        self.n_hits = int(batch.hit_offset[-1])

    def run(self):
        """Enqueue every queue after the current stream's work; the current
        stream then waits for all of them."""
        main = torch.cuda.current_stream(self.device)
        start = torch.cuda.Event()
        start.record(main)
        ends = []
        for p in self.parts:
            p["stream"].wait_event(start)
            with torch.cuda.stream(p["stream"]):
                p["tracker"].track(p["hits"], p["out"], self.form)
                e = torch.cuda.Event()
                e.record(p["stream"])
                ends.append(e)
        for e in ends:
            main.wait_event(e)

    def check(self):
        """Synchronise every queue; (status, tracklets) of each."""
        res = []
        for p in self.parts:
            with torch.cuda.stream(p["stream"]):
                res.append(p["tracker"].result())
        return res

    def time_ms(self, reps=2):
        """Milliseconds per pass over the whole batch (HIP events on the
        current stream around the queues' work)."""
        main = torch.cuda.current_stream(self.device)
        self.run()
        self.check()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize(self.device)
        e0.record(main)
        for _ in range(reps):
            self.run()
        e1.record(main)
        torch.cuda.synchronize(self.device)
        for st, _ in self.check():
            if st != 0:
                raise RuntimeError(f"catpc status {st}")
        return e0.elapsed_time(e1) / reps

    def close(self):
        for p in self.parts:
            p["tracker"].close()
        self.parts = []
