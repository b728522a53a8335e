"""Autotuner for the launch shape of the batched chain.

A joint grid over the tracklet kernel's register fit, resident waves per CU
then a coordinate search over the other catpc_tuning
fields (grid-bin occupancy, block sizes, row chunks, LDS staging), timing the replayed hipGraph with HIP
events on the caller's stream.  The result never changes the output (the
kernels' results do not depend on these values); it is written to a JSON cache
keyed by the device architecture, which bench.py and the serving loop read.

    python -m paper_1712_09430_amd.autotune --workload batch64 --out paper_1712_09430_amd/tuning_gfx950.json
"""
import argparse
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tuning_gfx950.json")

# Searched jointly first: how many waves the tracklet kernel keeps resident
# depends on its register fit.
JOINT = {
    "tc_sync": [0, 1],
    "tc_occupancy": [0, 5, 6, 8],
    "tc_waves_per_cu": [8, 12, 16, 20, 24, 32],
}
# Then one coordinate at a time.
SPACE = {
    "tc_xcd": [0, 1],
    "tc_block": [64, 128, 256],
    "bin_hits": [0.5, 1.0, 2.0, 4.0, 8.0],
    "nf_rows": [1, 2, 4, 8, 16],
    "nf_lds_kb": [0, 16, 32, 48, 64],
    "nf_block": [64, 128, 256],
}


def cached_tuning(arch=None, path=DEFAULT_CACHE):
    """The autotuner's result for this device architecture (dict), or None."""
    if not os.path.exists(path):
        return None
    if arch is None:
        import torch
        arch = torch.cuda.get_device_properties(0).gcnArchName
    cache = json.load(open(path))
    if cache.get("arch", "").split(":")[0] != arch.split(":")[0]:
        return None
    return cache["tuning"]


def time_config(tracker, hits, out, tuning, reps=5):
    import torch
    tracker.set_tuning(tuning)
    stream = torch.cuda.current_stream()
    tracker.track(hits, out)
    tracker.result()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        tracker.track(hits, out)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    st, _ = tracker.result()
    if st != 0:
        raise RuntimeError(f"catpc status {st}")
    times.sort()
    return times[len(times) // 2]


def tune(tracker, hits, out, passes=2, log=print):
    from . import catpc as C
    t = C.catpc_get_tuning(tracker.ctx)
    cur = {f: getattr(t, f) for f, _ in C.catpc_tuning._fields_}
    best_ms = time_config(tracker, hits, out, cur)
    log(f"[autotune] start {cur} {best_ms:.3f} ms")
    trials = []
    base = dict(cur)
    for sync in JOINT["tc_sync"]:
        for occ in JOINT["tc_occupancy"]:
            for waves in JOINT["tc_waves_per_cu"]:
                if occ and waves < 4 * occ - 8:
                    continue  # fewer resident waves than the occupancy variant is for
                cand = dict(base, tc_sync=sync, tc_occupancy=occ, tc_waves_per_cu=waves)
                if cand == cur:
                    continue
                ms = time_config(tracker, hits, out, cand)
                trials.append((cand, ms))
                log(f"[autotune] sync={sync} occupancy={occ} waves/CU={waves}: {ms:.3f} ms")
                if ms < best_ms * 0.99:
                    best_ms, cur = ms, cand
    for _ in range(passes):
        changed = False
        for field, values in SPACE.items():
            for v in values:
                if v == cur[field]:
                    continue
                cand = dict(cur, **{field: v})
                ms = time_config(tracker, hits, out, cand)
                trials.append((cand, ms))
                log(f"[autotune] {field}={v}: {ms:.3f} ms")
                if ms < best_ms * 0.99:
                    best_ms, cur, changed = ms, cand, True
        if not changed:
            break
    tracker.set_tuning(cur)
    return cur, best_ms, trials


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="batch64")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--out", default=DEFAULT_CACHE)
    args = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    import torch

    import bench
    from .tracker import DeviceHits, Tracker
    batch, desc = bench.workload(args.workload, args.seed)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)
    hits = DeviceHits(batch.y, batch.z, batch.row, batch.hit_offset, "cuda:0")
    tr = Tracker(batch.row_x, hits.n_hits, hits.n_sectors)
    start = cached_tuning()
    if start is not None:  # continue from the last result
        tr.set_tuning(start)
    out = tr.output(hits)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    best, ms, trials = tune(tr, hits, out, log=log)
    arch = torch.cuda.get_device_properties(0).gcnArchName
    res = {"arch": arch, "workload": desc, "n_hits": hits.n_hits, "best_ms": ms, "tuning": best,
           "trials": [{"tuning": t, "ms": m} for t, m in trials]}
    with open(args.out, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps({"best": best, "ms": ms}))


if __name__ == "__main__":
    main()
