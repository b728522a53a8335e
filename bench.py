"""Benchmark of the sector-tracking hot path on one MI355X.

One step = the whole hot path (row index + grids, neighbour finding, link
cleaning + start hits, tracklet construction) over one batch of seeded
synthetic events, inputs already resident in HBM.  Default workload: 64
events with multiplicities log-uniform from 20 to 10^4 tracks (2304 uneven
sectors), the batched form (fixed chain of persistent launches replayed as a
hipGraph).  The same batch is also timed in the plain form (the stages
launched sector by sector), and the oracle is timed on a bounded sample of
the same batch on the host cores.

Prints one JSON line.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TPC hits/s (CA+tracklet fit) batched vs plain on 1 GPU; p99 event latency"
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
# Algorithmic work per unit ("Measurement"):
NF_BYTES_PER_HIT = 16.0        # y, z in (8 B) + up, down link out (8 B)
FLOPS_PER_TRANSPORT = 75.0     # binary32 operations of one helix transport incl. covariance
FLOPS_PER_UPDATE = 39.0        # two scalar Kalman updates
FLOPS_PER_SEARCH = 6.0         # the two gate widths
FLOPS_PER_CANDIDATE = 5.0      # residuals and squared distance of a gated cluster


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "traffic_batch64.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1712_09430_amd", "csrc", "kernels.hip")


def kernels_digest():
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def profiled_traffic(workload_name, tuning):
    """HBM bytes per launch from the committed counter summary (rocprofv3
    FETCH_SIZE and WRITE_SIZE passes, scaled by a copy kernel of known size),
    valid only for the kernel source, workload and launch shape it was taken
    with; {} otherwise."""
    if not os.path.exists(TRAFFIC_PROFILE):
        return {}
    rec = None
    for line in open(TRAFFIC_PROFILE):
        line = line.strip()
        if line.startswith("<!-- traffic ") and line.endswith("-->"):
            rec = json.loads(line[len("<!-- traffic "):-3])
    shape = lambda t: {k: v for k, v in t.items() if k != "use_graph"}  # graph replay launches the same kernels
    if (rec is None or rec.get("kernels_sha256") != kernels_digest() or rec.get("workload") != workload_name
            or shape(rec.get("tuning", {})) != shape(tuning)):
        return {}
    return rec["per_launch"]


def workload(name, seed):
    import synth
    if name == "batch64":
        b = synth.batch_workload(seed=seed, n_events=64)
        desc = (f"batch64: 64 events, multiplicity floor(exp(U(ln 20, ln 1e4))) tracks ({sum(b.multiplicity)} "
                f"tracks), 36 sectors x 159 pad rows each ({b.n_sectors} sectors), Bz 0.5 T, pT log-uniform "
                f"0.2-10 GeV, |eta|<0.9, smear 0.1 cm, 10% noise")
    elif name == "event":
        b = synth.event_workload(seed=seed, n_tracks=10000)
        desc = "event: one central-heavy-ion-like event, 10k tracks over 36 sectors x 159 pad rows"
    elif name == "sector":
        b = synth.sector_workload(seed=seed, n_tracks=200)
        desc = "sector: one sector, 200 tracks, 159 pad rows"
    else:
        raise SystemExit(f"unknown workload {name}")
    return b, desc


def cpu_baseline(batch, target_hits, cores):
    """The oracle (binary32 mode, whole sector path) on a bounded sample of the
    workload's sectors, sectors spread over `cores` threads (ctypes releases
    the GIL)."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    sizes = np.diff(batch.hit_offset)
    order = np.argsort(-sizes, kind="stable")
    # every k-th sector by size so the sample has the workload's size mix
    k = max(1, int(math.ceil(batch.n_hits / max(target_hits, 1))))
    pick = sorted(order[::k].tolist())
    n = int(sizes[pick].sum())
    p = oracle.Params()
    oracle.lib()

    def run(s):
        sec = batch.sector(s)
        oracle.track_sector(sec["y"], sec["z"], sec["row"], batch.row_x, p, "f32")

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as ex:
        list(ex.map(run, pick))
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "hits/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(pick)} of {batch.n_sectors} sectors (every {k}th by size), {n} hits, whole sector "
                      f"path in binary32, sectors spread over {cores} threads; {dt:.2f} s wall",
            "seconds": dt}


def serving_leg(args, tuning, log):
    """Poisson stream of events (multiplicities as in the batch workload) through
    the continuous-batching server; latency from arrival to results in host
    memory (H2D, the hot path and D2H included)."""
    import synth
    from paper_1712_09430_amd import serve
    log(f"[bench] serving: {args.serve_events} events at {args.serve_rate:g} Hz")
    pool = synth.event_pool(seed=2, n_events=64)
    rng = np.random.default_rng(3)
    order = rng.integers(0, len(pool), args.serve_events)
    arrival = serve.poisson_arrivals(args.serve_events, args.serve_rate, seed=4)
    src = serve.EventStream(pool, order, arrival, pool[0].row_x)
    res = serve.serve(src, tuning=tuning, warmup_events=args.serve_warmup)
    log(f"[bench] serving: p50 {res['p50_ms']:.3f} ms, p99 {res['p99_ms']:.3f} ms, {res['hits_per_s']:.4g} hits/s, "
        f"{res['batches']} batches, {res['slots']} slots")
    # the same stream with every event waiting from the start: the server's
    # saturated throughput (H2D, hot path and D2H of overlapping batches)
    sat = serve.serve(src, tuning=tuning, warmup_events=0, realtime=False)
    log(f"[bench] serving saturated: {sat['hits_per_s']:.4g} hits/s, {sat['batches']} batches")
    return {"p50_ms": res["p50_ms"], "p99_ms": res["p99_ms"], "hits_per_s": res["hits_per_s"],
            "events": res["n_events"], "warmup_events": args.serve_warmup, "rate_hz": args.serve_rate,
            "batches": res["batches"], "mean_batch_events": res["mean_batch_events"], "slots": res["slots"],
            "hbm_budget_gib": res["hbm_budget_bytes"] / 2**30,
            "slot_footprint_gib": res["slot_footprint_bytes"] / 2**30,
            "latency": "arrival to results in host memory (H2D + hot path + D2H)",
            "saturated_hits_per_s": sat["hits_per_s"], "saturated_batches": sat["batches"],
            "late_fetches": res["late_fetches"],
            "mean_event_hits": float(src.ev_hits.mean())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch64")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--cpu-hits", type=float, default=6e6, help="oracle sample size for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tuning", default="auto",
                    help="'auto' (the autotuner's cache for this architecture, if present), 'default', or a JSON "
                         "file with catpc tuning values")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="launch the chain directly (for counter runs)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="before the timed region, one device copy of this many MiB (calibrates HBM counters)")
    ap.add_argument("--serve-events", type=int, default=2200, help="serving leg: events in the stream (0: skip)")
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--serve-rate", type=float, default=1000.0, help="serving leg: Poisson arrival rate, Hz")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the hot path shards by event with no "
                                   "exchange (see DESIGN.md), multi-GPU runs are not part of this build",
                          "n_gpus": args.gpus}))
        raise SystemExit(2)

    import torch

    from paper_1712_09430_amd import catpc as C
    from paper_1712_09430_amd.tracker import DeviceHits, Tracker

    log = (lambda *a: None) if args.quiet else (lambda *a: print(*a, file=sys.stderr, flush=True))
    log(f"[bench] generating workload {args.workload} seed {args.seed}")
    batch, desc = workload(args.workload, args.seed)
    dev = "cuda:0"
    torch.cuda.init()
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(stream)
    hits = DeviceHits(batch.y, batch.z, batch.row, batch.hit_offset, dev)
    tr = Tracker(batch.row_x, hits.n_hits, hits.n_sectors, device=dev)
    tuning_src = "library defaults"
    if args.tuning == "auto":
        from paper_1712_09430_amd import autotune
        cached = autotune.cached_tuning()
        if cached is not None:
            tr.set_tuning(cached)
            tuning_src = "autotuner cache " + os.path.basename(autotune.DEFAULT_CACHE)
    elif args.tuning != "default":
        tr.set_tuning(json.load(open(args.tuning)))
        tuning_src = args.tuning
    if args.no_graph:
        tr.set_tuning({"use_graph": 0})
    t = C.catpc_get_tuning(tr.ctx)
    tuning = {f: getattr(t, f) for f, _ in C.catpc_tuning._fields_}
    if args.copy_mib > 0:
        # counter calibration: one elementwise kernel that reads copy_mib MiB
        # and writes copy_mib MiB, its source pushed out of the caches first
        n = args.copy_mib * (1 << 20) // 4
        src = torch.full((n,), 1.0, dtype=torch.float32, device=dev)
        evict = torch.zeros(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        log(f"[bench] calibration kernel: {args.copy_mib} MiB read, {args.copy_mib} MiB written")
        del src, evict, dst
    out = tr.output(hits)
    log(f"[bench] {hits.n_hits} hits in {hits.n_sectors} sectors; warmup {args.warmup}")

    for _ in range(args.warmup):
        tr.track(hits, out)
    st, n_trk = tr.result()
    if st != C.CATPC_OK:
        raise SystemExit(f"catpc status {st}: {C.catpc_last_error()}")

    # timed batched steps
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        tr.track(hits, out)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = e0.elapsed_time(e1) / args.steps
    st, n_trk = tr.result()
    if st != C.CATPC_OK:
        raise SystemExit(f"catpc status {st}: {C.catpc_last_error()}")
    value = hits.n_hits / (ms_step * 1e-3)
    log(f"[bench] batched: {ms_step:.3f} ms/step, {value:.4g} hits/s, {n_trk} tracklets (wall {wall:.3f} s)")

    # per-stage times (HIP events between the stages, on this stream)
    stage = np.median(np.stack([tr.stage_times(hits, out) for _ in range(5)]), axis=0)
    work = tr.work_counts()
    stages = {name: float(v) for name, v in zip(C.STAGES, stage)}
    log("[bench] stages ms: " + ", ".join(f"{k} {v:.3f}" for k, v in stages.items()))

    flops = (work[0] * FLOPS_PER_TRANSPORT + work[1] * FLOPS_PER_UPDATE + work[3] * FLOPS_PER_SEARCH +
             work[2] * FLOPS_PER_CANDIDATE)
    tc_ms = stages["tracklets"]
    nf_ms = stages["neighbours"]
    rl_tc = {"kernel": "k_tracklets", "bound": "alu", "achieved": flops / (tc_ms * 1e-3) / 1e12,
             "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "traffic": None, "launch_ms": tc_ms,
             "algorithmic_flops": float(flops), "work_counts": work.tolist()}
    rl_tc["frac"] = rl_tc["achieved"] / rl_tc["peak"]
    nf_bytes = NF_BYTES_PER_HIT * hits.n_hits
    rl_nf = {"kernel": "k_neighbours", "bound": "hbm", "achieved": nf_bytes / (nf_ms * 1e-3) / 1e9,
             "peak": HBM_PEAK_GBS, "unit": "GB/s", "traffic": None, "launch_ms": nf_ms,
             "algorithmic_bytes": nf_bytes}
    rl_nf["frac"] = rl_nf["achieved"] / rl_nf["peak"]
    traffic = profiled_traffic(args.workload, tuning)
    for rl in (rl_tc, rl_nf):
        t = traffic.get(rl["kernel"])
        if t:
            rl["traffic"] = t["fetch_bytes"] + t["write_bytes"]
            rl["traffic_fetch"], rl["traffic_write"] = t["fetch_bytes"], t["write_bytes"]
            rl["traffic_source"] = os.path.relpath(TRAFFIC_PROFILE, ROOT)
    dominant = rl_tc if tc_ms >= nf_ms else rl_nf

    # plain form: the same stages launched sector by sector
    plain = None
    if args.plain_steps > 0:
        tr.track(hits, out, "plain")
        tr.result()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.plain_steps):
            tr.track(hits, out, "plain")
        e1.record(stream)
        torch.cuda.synchronize()
        st, n2 = tr.result()
        pms = e0.elapsed_time(e1) / args.plain_steps
        plain = {"hits_per_s": hits.n_hits / (pms * 1e-3), "ms_per_step": pms, "steps": args.plain_steps,
                 "launches_per_step": 8 * hits.n_sectors + 1, "status": int(st), "n_tracklets": n2}
        log(f"[bench] plain: {pms:.3f} ms/step, {plain['hits_per_s']:.4g} hits/s")

    serving = None
    if args.serve_events > 0:
        serving = serving_leg(args, tuning, log)

    cpu = None
    if not args.no_cpu_baseline:
        cores = min(16, os.cpu_count() or 1)
        log(f"[bench] oracle on a sample, {cores} threads")
        cpu = cpu_baseline(batch, args.cpu_hits, cores)
        log(f"[bench] oracle: {cpu['value']:.4g} hits/s")

    res = {"metric": METRIC, "value": value, "unit": "hits/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic (seeded helix events, no recorded data)",
           "config": {"workload": desc, "n_hits": hits.n_hits, "n_sectors": hits.n_sectors,
                      "n_tracklets": n_trk, "seed": args.seed, "form": "batched: fixed launch chain over all "
                      "sectors, persistent tracklet kernel, hipGraph replay", "parallelism": "single GPU",
                      "tuning": tuning, "tuning_source": tuning_src},
           "plain": plain, "batched_over_plain": (value / plain["hits_per_s"]) if plain else None,
           "serving": serving, "stages_ms": stages, "roofline": {k: v for k, v in dominant.items() if k != "kernel"} |
           {"kernel": dominant["kernel"]}, "rooflines": {"k_tracklets": rl_tc, "k_neighbours": rl_nf},
           "cpu_baseline": cpu}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
