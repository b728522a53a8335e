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
# Algorithmic work per unit (binary32 operations of the formulas, division and square root count 1):
NF_BYTES_PER_HIT = 16.0        # y, z in (8 B) + up, down link out (8 B)
# the other per-hit stages, algorithmic bytes per hit (the method's own data, not this layout's):
GRID_BYTES_PER_HIT = 24.0      # y, z, row in (12 B); sorted y, z and the permutation out (12 B)
CLEAN_BYTES_PER_HIT = 36.0     # cleaning: links and the partners' back links in, cleaned links out (24 B);
                               # start hits: cleaned links in, start bits out (about 12 B)
ROWIDX_BYTES_PER_HIT = 4.0     # row in
FLOPS_PER_TRANSPORT = 75.0     # binary32 operations of one helix transport incl. covariance
FLOPS_PER_UPDATE = 39.0        # two scalar Kalman updates
FLOPS_PER_SEARCH = 6.0         # the two gate widths
FLOPS_PER_CANDIDATE = 5.0      # residuals and squared distance of a gated cluster


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "traffic_batch64.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1712_09430_amd", "csrc", "kernels.hip")


def kernels_digest():
    """SHA-256 of the kernel source followed by the library's build flags."""
    from paper_1712_09430_amd import build as B
    h = hashlib.sha256()
    with open(KERNEL_SOURCE, "rb") as f:
        h.update(f.read())
    h.update(" ".join(B.FLAGS).encode())
    return h.hexdigest()


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


DEAD_BAND = (70, 8)  # pad rows without clusters in the merging leg's second batch
# binary64 operations of the merging's chi^2 pass: one row step of the transport (50 for the state
# and the Jacobian, 190 for F C F^T over the structurally nonzero entries of F: 55 + 40 products and
# as many additions), and per pair the summed covariance, Cholesky factorisation, forward
# substitution and the difference (110)
MERGE_FLOPS_PER_STEP = 240
MERGE_FLOPS_PER_PAIR = 110
PEAK_FP64_TFLOPS = 78.6
# binary64 operations of the full refit, counted the same way: a state-only transport from the
# tracklet's first row to the track's first hit (33), a row step with the covariance (240), and a
# 2-d update (residuals, 2x2 inverse, gain, state, covariance and chi^2: 135)
REFIT_FLOPS_TRANSPORT = 33
REFIT_FLOPS_STEP = 240
REFIT_FLOPS_UPDATE = 135


def refit_work(batch, out, n_trk, tnp, fn):
    """Row steps of the refit's finished fits, from the tracks, their
    tracklets and the hits: state-only transports (tracklet first row to the
    first hit's row), transports with covariance (first to last hit's row),
    and updates (hits used, from ndf = 2 used - 5)."""
    ok = fn["flags"] == 1
    toff = tnp["track_offset"]
    sec = np.repeat(np.arange(len(toff) - 1), np.diff(toff))
    nh, h0 = tnp["track_n_hits"], tnp["track_hit_offset"]
    a = batch.hit_offset[sec]
    r_first = batch.row[a + tnp["track_hits"][h0]]
    r_last = batch.row[a + tnp["track_hits"][h0 + nh - 1]]
    slot = out.tracklet_offset.cpu().numpy()[sec] + tnp["track_tracklet"]
    start = out.first_row[:n_trk].cpu().numpy()[slot]
    used = (fn["ndf"] + 5) // 2
    return (int(np.sum((r_first - start)[ok])), int(np.sum((r_last - r_first)[ok])), int(np.sum(used[ok])))


def merge_leg(tr, hits, out, tracks, fits, n_tracks, stream, reps=5):
    """Time the segment merging (HIP events on `stream`) and count its links."""
    import torch
    merges = tr.merges_output(tracks)
    tr.merge(hits, out, tracks, fits, merges)
    torch.cuda.synchronize()
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s0.record(stream)
    for _ in range(reps):
        tr.merge(hits, out, tracks, fits, merges)
    s1.record(stream)
    torch.cuda.synchronize()
    mn = merges.numpy(n_tracks)
    pairs, steps = tr.merge_counts()
    ms = s0.elapsed_time(s1) / reps
    flops = MERGE_FLOPS_PER_STEP * steps + MERGE_FLOPS_PER_PAIR * pairs
    return {"ms": ms, "tracks": int(n_tracks), "links": int(np.sum(mn["next"] >= 0)),
            "chains": int(np.sum((mn["next"] >= 0) & (mn["prev"] < 0))),
            "candidate_pairs": int(pairs), "transport_steps": int(steps),
            "fp64_tflops": flops / (ms * 1e-3) / 1e12, "fp64_peak_tflops": PEAK_FP64_TFLOPS,
            "what": "segment merging inside each sector: straight-line window, transported 5x5 covariance, "
                    "chi^2 of the two states, mutual best link (binary64)"}


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


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def peak_probes(torch, C, dev, stream, log):
    """Achievable peaks on this GPU with the library's own probes: a 4 GiB
    device copy (bytes read + written per second) and 8 independent FMA chains
    per thread over 2^20 threads (binary32, non-packed)."""
    n = 4 << 30
    src = torch.empty(n // 4, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    sp = stream.cuda_stream
    C.catpc_probe_copy(src.data_ptr(), dst.data_ptr(), n, sp)  # warm
    reps = 5
    e0.record(stream)
    for _ in range(reps):
        C.catpc_probe_copy(src.data_ptr(), dst.data_ptr(), n, sp)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    threads, iters = 1 << 20, 4096
    out = torch.empty(threads, dtype=torch.float32, device=dev)
    C.catpc_probe_fma(out.data_ptr(), threads, iters, sp)
    e0.record(stream)
    for _ in range(reps):
        C.catpc_probe_fma(out.data_ptr(), threads, iters, sp)
    e1.record(stream)
    torch.cuda.synchronize()
    fma_tflops = 16.0 * threads * iters * reps / (e0.elapsed_time(e1) * 1e-3) / 1e12
    log(f"[bench] probes: copy {copy_gbs:.0f} GB/s, FP32 FMA {fma_tflops:.1f} TFLOP/s")
    return {"copy_gbs": copy_gbs, "fma_tflops": fma_tflops,
            "copy": "4 GiB device copy, 16 B per lane, bytes read + written",
            "fma": "2^20 threads x 4096 iterations x 8 independent binary32 FMA chains (non-packed)"}


def truth_pulls(b, t, valid):
    """Pulls (p - p_true) / sqrt(C_ii) of y, z, sin phi, tan lambda, q/pT at
    x_ref over truth-matched tracklets: at least 90 % of the hits from one
    generated track, whose own hit sits in the tracklet's first row (the
    generator's true position there is the truth at x_ref)."""
    tr0 = b.tracks[0]
    names = ("y", "z", "sinphi", "tanl", "qpt")
    rows = []
    for k in np.flatnonzero(valid):
        rh = t["row_hit"][k][:b.n_rows]
        hits = rh[rh >= 0]
        lab = b.label[hits]
        vals, cnt = np.unique(lab, return_counts=True)
        L = vals[cnt.argmax()]
        h = rh[t["first_row"][k]]
        if L < 0 or cnt.max() < 0.9 * len(hits) or h < 0 or b.label[h] != L:
            continue
        truth = np.array([b.truth["y_true"][h], b.truth["z_true"][h], b.truth["sinphi_true"][h],
                          math.sinh(tr0["eta"][L]), tr0["q"][L] / tr0["pt"][L]])
        var = t["cov"][k][[0, 2, 5, 9, 14]].astype(np.float64)
        if np.all(var > 0):
            rows.append((t["param"][k].astype(np.float64) - truth) / np.sqrt(var))
    p = np.array(rows).reshape(-1, 5)
    return {n: {"mean": float(p[:, i].mean()), "rms": float(np.sqrt((p[:, i] ** 2).mean())), "n": len(p)}
            for i, n in enumerate(names)} | {"matched_tracklets": len(p)}


def precision_leg(torch, tuning, log):
    """The precision form (binary32 filter; binary64 covariance refit only for
    tracklets whose binary32 covariance fails the SPD check) on the
    one-sector workload (200 tracks) and on the same sector with precise
    clusters (smear and fit error 3e-4 cm, where binary32 pivots do fail):
    failures, refits, and pulls over truth-matched tracklets.  The GPU
    tracklets are kept for the oracle leg's binary64 parameter check."""
    import synth
    from paper_1712_09430_amd import catpc as C
    from paper_1712_09430_amd.tracker import DeviceHits, Tracker
    rep, keep = {}, {}
    for name, seed, sigma in (("sector", 1, 0.1), ("sector_precise_clusters", 11, 3e-4)):
        b = synth.sector_workload(seed=seed, n_tracks=200, truth=True, sigma=sigma)
        hits = DeviceHits(b.y, b.z, b.row, b.hit_offset, "cuda:0")
        r = {"workload": f"sector: one sector, 200 tracks, 159 pad rows, seed {seed}, cluster smear and fit "
                         f"error {sigma:g} cm", "n_hits": hits.n_hits}
        for prec in (0, 1):
            p = C.catpc_default_params()
            p.precision = prec
            p.sigma_y = p.sigma_z = sigma
            tr = Tracker(b.row_x, hits.n_hits, hits.n_sectors, params=p)
            tr.set_tuning(dict(tuning, use_graph=0))
            out = tr.output(hits)
            tr.track(hits, out)
            st, n = tr.result()
            t = out.tracklets_numpy(n)
            fl = t["flags"]
            valid = (fl & C.FLAG_VALID) != 0
            r[f"precision_{prec}"] = {"tracklets": int(n), "valid": int(valid.sum()),
                                      "spd_failures": int(((fl & C.FLAG_SPD_FAIL) != 0).sum()),
                                      "refits": int(((fl & C.FLAG_REFIT64) != 0).sum()),
                                      "pulls_truth_matched": truth_pulls(b, t, valid)}
            keep[(name, prec)] = (b, t, p)
            tr.close()
        rep[name] = r
        log(f"[bench] precision {name}: SPD failures {r['precision_0']['spd_failures']}, "
            f"refits {r['precision_1']['refits']} of {r['precision_1']['tracklets']} tracklets")
    rep["pull_definition"] = ("(p - p_true) / sqrt(C_ii) at x_ref over valid tracklets with >= 90 % of their hits "
                              "from one generated track whose own hit is in the tracklet's first row")
    return rep, keep


STRICT_ABS = np.array([1e-3, 1e-3, 0.0, 0.0, 0.0])
STRICT_REL = np.array([0.0, 0.0, 1e-4, 1e-4, 1e-4])
STRICT_FLOOR = np.array([1.0, 1.0, 1.0, 1.0, 0.1])


def parameter_check(items):
    """ORACLE LEG: binary32 GPU parameters against the binary64 oracle refit of
    the same hits (y, z within 1e-3 cm; sin phi, tan lambda within 1e-4 of
    max(|ref|, 1); q/pT within 1e-4 of max(|ref|, 0.1)).  items: (y, z,
    row_x, tracklet dict, params) per sector.  Returns the fraction of
    compared tracklets with all five inside, the per-parameter maximum
    deviation, and the q/pT values outside (count, largest deviation in units
    of their binary64 standard error)."""
    import oracle
    devs, sigq = [], []
    for y, z, row_x, t, p in items:
        op = oracle.Params(bz=p.bz, sigma_y=p.sigma_y, sigma_z=p.sigma_z)
        if len(t["flags"]) == 0:
            continue
        r = oracle.refit(y, z, row_x, t["row_hit"][:, :len(row_x)], t["start_row"], op, "f64")
        good = ((t["flags"] & 1) != 0) & ((r["flags"] & 1) != 0)
        devs.append(np.abs(t["param"][good].astype(np.float64) - r["param"][good]) /
                    (STRICT_ABS + STRICT_REL * np.maximum(np.abs(r["param"][good]), STRICT_FLOOR)))
        sigq.append(np.abs(t["param"][good, 4].astype(np.float64) - r["param"][good, 4]) /
                    np.sqrt(r["cov"][good, 14]))
    d = np.concatenate(devs) if devs else np.zeros((0, 5))
    sq = np.concatenate(sigq) if sigq else np.zeros(0)
    inside = np.all(d <= 1.0, axis=1)
    outq = d[:, 4] > 1.0
    return {"tracklets": int(len(d)), "fraction_strict": float(inside.mean()) if len(d) else None,
            "max_over_bound": {k: float(d[:, i].max()) if len(d) else None
                               for i, k in enumerate(("y", "z", "sinphi", "tanl", "qpt"))},
            "qpt_outside": int(outq.sum()),
            "qpt_outside_max_dev_over_sigma": float(sq[outq].max()) if outq.any() else None,
            "bound": "y, z 1e-3 cm; sin phi, tan lambda 1e-4 max(|ref|, 1); q/pT 1e-4 max(|ref|, 0.1); "
                     "max_over_bound = largest deviation / its bound"}


def scheduling_leg(batch, tuning, hits_total, log):
    """The paper's scheduling schemes for the per-sector form on this GPU
    (Sec. 3.1: sectors over 8 queues; Sec. 3.2: several tracker instances by
    event), beside the single persistent batched chain."""
    from paper_1712_09430_amd.schedule import Queues
    out = {}
    for name, q, by, form, reps in (("plain_8_queues_by_sector", 8, "sector", "plain", 1),
                                    ("plain_4_instances_by_event", 4, "event", "plain", 1),
                                    ("batch_2_instances_by_event", 2, "event", "batch", 3),
                                    ("batch_4_instances_by_event", 4, "event", "batch", 3)):
        Q = Queues(batch, q, by=by, form=form, tuning=tuning)
        ms = Q.time_ms(reps)
        Q.close()
        out[name] = {"ms_per_step": ms, "hits_per_s": hits_total / (ms * 1e-3)}
        log(f"[bench] scheduling {name}: {ms:.2f} ms/step")
    return out


def config_lines(torch, tuning, seed, log, reps=20, plain_reps=5):
    """The single-sector workload (200 tracks) and the full central event
    (10k tracks, 36 sectors), each in the batched form (graph replay, median
    of `reps` HIP-event-timed steps after 3 warm-up steps) and in the plain
    form (per-sector launches, median of `plain_reps`)."""
    from paper_1712_09430_amd.tracker import DeviceHits, Tracker
    stream = torch.cuda.current_stream()
    res = {}
    for name in ("sector", "event"):
        b, desc = workload(name, seed)
        hits = DeviceHits(b.y, b.z, b.row, b.hit_offset, "cuda:0")
        tr = Tracker(b.row_x, hits.n_hits, hits.n_sectors, tuning=tuning)
        out = tr.output(hits)
        line = {"workload": desc, "n_hits": int(hits.n_hits), "n_sectors": int(hits.n_sectors)}
        for form, k in (("batch", reps), ("plain", plain_reps)):
            for _ in range(3):
                tr.track(hits, out, form)
            st, n = tr.result()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(k + 1)]
            ev[0].record(stream)
            for i in range(k):
                tr.track(hits, out, form)
                ev[i + 1].record(stream)
            torch.cuda.synchronize()
            ms = float(np.median([ev[i].elapsed_time(ev[i + 1]) for i in range(k)]))
            line[form] = {"ms_per_step": ms, "hits_per_s": hits.n_hits / (ms * 1e-3), "steps": k,
                          "n_tracklets": int(n), "status": int(st)}
            log(f"[bench] {name} {form}: {ms:.3f} ms/step, {line[form]['hits_per_s']:.4g} hits/s")
        line["batched_over_plain"] = line["batch"]["hits_per_s"] / line["plain"]["hits_per_s"]
        res[name] = line
        tr.close()
        del hits, out
    return res


LINEARITY_TRACKS = (250, 500, 1000, 2000, 4000, 8000, 16000)


def linearity_leg(torch, tuning, seed, log, reps=10):
    """Tracking time against input size (the tracking follows at most one
    hypothesis per hit, so its time grows about linearly with the hits):
    single events of increasing multiplicity through the batched chain,
    median of `reps` HIP-event-timed calls each; a least-squares line
    t = a + b * hits and the log-log slope over the larger half."""
    import synth
    from paper_1712_09430_amd.tracker import DeviceHits, Tracker
    dev = "cuda:0"
    stream = torch.cuda.current_stream()
    evs = [synth.event_workload(seed=seed, n_tracks=n) for n in LINEARITY_TRACKS]
    hmax = max(int(e.n_hits) for e in evs)
    tr = Tracker(evs[0].row_x, hmax, max(e.n_sectors for e in evs), device=dev, tuning=tuning)
    pts = []
    for n, e in zip(LINEARITY_TRACKS, evs):
        hits = DeviceHits(e.y, e.z, e.row, e.hit_offset, dev)
        out = tr.output(hits)
        for _ in range(2):
            tr.track(hits, out)
        tr.result()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        ev[0].record(stream)
        for k in range(reps):
            tr.track(hits, out)
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        ms = float(np.median([ev[k].elapsed_time(ev[k + 1]) for k in range(reps)]))
        pts.append((int(hits.n_hits), ms))
        log(f"[bench] linearity: {n} tracks, {hits.n_hits} hits, {ms:.3f} ms")
        del hits, out
    tr.close()
    h = np.array([p[0] for p in pts], float)
    t = np.array([p[1] for p in pts], float)
    b, a = np.polyfit(h, t, 1)
    r2 = 1.0 - np.sum((t - (a + b * h)) ** 2) / np.sum((t - t.mean()) ** 2)
    big = h >= np.median(h)
    slope = float(np.polyfit(np.log(h[big]), np.log(t[big]), 1)[0])
    res = {"tracks": list(LINEARITY_TRACKS), "hits": [int(x) for x in h], "ms": [float(x) for x in t],
           "fit_ms": {"intercept": float(a), "per_mhit": float(b * 1e6)}, "r2": float(r2),
           "loglog_slope_upper_half": slope,
           "what": "single events through the batched chain; time vs hits, least-squares line and log-log slope"}
    log(f"[bench] linearity: t = {a:.3f} ms + {b * 1e6:.3f} ms/Mhit, R^2 {r2:.4f}, log-log slope {slope:.3f}")
    return res


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
    from paper_1712_09430_amd import autotune
    stun = autotune.cached_serve_tuning() if args.tuning == "auto" else None
    source = "autotuner serving result" if stun else "the batch tuning"
    stun = stun or tuning
    res = serve.serve(src, tuning=stun, warmup_events=args.serve_warmup)
    log(f"[bench] serving: p50 {res['p50_ms']:.3f} ms, p99 {res['p99_ms']:.3f} ms, {res['hits_per_s']:.4g} hits/s, "
        f"{res['batches']} batches, {res['slots']} slots, peak in flight "
        f"{res['peak_in_flight_bytes'] / 2**20:.0f} MiB, {res['deferred_events']} deferred")
    # the same stream (first 3000 events) under a budget of twice the largest event's footprint: the
    # budget, not the slot count, then decides admissions
    n_tight = min(3000, args.serve_events)
    src_t = serve.EventStream(pool, order[:n_tight], arrival[:n_tight], pool[0].row_x)
    tight_budget = 2 * res["largest_event_footprint_bytes"]
    tight = serve.serve(src_t, tuning=stun, warmup_events=min(args.serve_warmup, n_tight // 10),
                        hbm_budget=tight_budget)
    log(f"[bench] serving, budget {tight_budget / 2**20:.0f} MiB: p50 {tight['p50_ms']:.3f} ms, "
        f"p99 {tight['p99_ms']:.3f} ms, {tight['slots']} slots, {tight['deferred_events']} deferred")
    # the same stream with every event waiting from the start: the server's
    # saturated throughput (H2D, hot path and D2H of overlapping batches)
    sat = serve.serve(src, tuning=stun, warmup_events=0, realtime=False)
    log(f"[bench] serving saturated: {sat['hits_per_s']:.4g} hits/s, {sat['batches']} batches")
    return {"p50_ms": res["p50_ms"], "p99_ms": res["p99_ms"], "hits_per_s": res["hits_per_s"],
            "events": res["n_events"], "warmup_events": args.serve_warmup, "rate_hz": args.serve_rate,
            "batches": res["batches"], "mean_batch_events": res["mean_batch_events"], "slots": res["slots"],
            "hbm_budget_gib": res["hbm_budget_bytes"] / 2**30,
            "slot_reserved_gib": res["slot_reserved_bytes"] / 2**30,
            "footprint_model": "per batch: input + 3 x input (internal) + outputs (links, start list, "
                               "estimated tracklet records)",
            "full_batch_footprint_gib": res["full_batch_footprint_bytes"] / 2**30,
            "largest_event_footprint_mib": res["largest_event_footprint_bytes"] / 2**20,
            "peak_in_flight_mib": res["peak_in_flight_bytes"] / 2**20,
            "deferred_events": res["deferred_events"],
            "tight_budget": {"budget_mib": tight_budget / 2**20, "events": tight["n_events"],
                             "slots": tight["slots"], "p50_ms": tight["p50_ms"], "p99_ms": tight["p99_ms"],
                             "hits_per_s": tight["hits_per_s"], "deferred_events": tight["deferred_events"],
                             "peak_in_flight_mib": tight["peak_in_flight_bytes"] / 2**20,
                             "what": "first 3000 events of the same stream, budget = twice the largest event's "
                                     "footprint"},
            "latency": "arrival to results in host memory (H2D + hot path + D2H)",
            "saturated_hits_per_s": sat["hits_per_s"], "saturated_batches": sat["batches"],
            "late_fetches": res["late_fetches"],
            "mean_event_hits": float(src.ev_hits.mean()),
            "tuning_source": source, "tuning_changes": {k: v for k, v in stun.items() if tuning.get(k) != v}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch64")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--plain-steps", type=int, default=5)
    ap.add_argument("--cpu-hits", type=float, default=3e7, help="oracle sample size for cpu_baseline (all threads)")
    ap.add_argument("--cpu-hits-1", type=float, default=1.5e6, help="oracle sample size on one thread")
    ap.add_argument("--cpu-hits-4", type=float, default=6e6, help="oracle sample size on four threads")
    ap.add_argument("--no-peaks", action="store_true", help="skip the copy and FMA peak probes")
    ap.add_argument("--no-precision", action="store_true", help="skip the precision-form report")
    ap.add_argument("--no-scheduling", action="store_true", help="skip the scheduling baselines")
    ap.add_argument("--no-linearity", action="store_true", help="skip the time-vs-hits check")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the one-sector and full-event lines (batched and plain)")
    ap.add_argument("--no-dead-band", action="store_true",
                    help="skip the merging leg's second batch (same events, 8 dead pad rows)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tuning", default="auto",
                    help="'auto' (the autotuner's cache for this architecture, if present), 'default', or a JSON "
                         "file with catpc tuning values")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="launch the chain directly (for counter runs)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="before the timed region, one device copy of this many MiB (calibrates HBM counters)")
    ap.add_argument("--serve-events", type=int, default=10500, help="serving leg: events in the stream (0: skip)")
    ap.add_argument("--serve-warmup", type=int, default=500)
    ap.add_argument("--serve-rate", type=float, default=1000.0, help="serving leg: Poisson arrival rate, Hz")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "only the one-GPU form is implemented: the hot path would shard by event "
                                   "with no exchange between GPUs, each GPU running this chain on its share",
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
            tuning_src = "autotuner cache " + os.path.basename(autotune.DEFAULT_CACHE) + (
                " (tuned on these kernels)" if autotune.cache_is_current() else
                " (tuned on an earlier kernel source)")
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
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    e0.record(stream)
    ev[0].record(stream)
    for k in range(args.steps):
        tr.track(hits, out)
        ev[k + 1].record(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = e0.elapsed_time(e1) / args.steps
    step_ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
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

    # tracklet selection after the hot path (graph replay, HIP events on this stream)
    tracks = tr.tracks_output(hits, out)
    tr.track(hits, out)
    tr.select(hits, out, tracks)
    n_tracks, n_track_hits = tr.select_result()
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s0.record(stream)
    for _ in range(5):
        tr.select(hits, out, tracks)
    s1.record(stream)
    torch.cuda.synchronize()
    sel = {"ms": s0.elapsed_time(s1) / 5, "tracks": n_tracks, "track_hits": n_track_hits,
           "what": "tracklet selection of the batch's tracklets (hit ownership by weight, min_hits kept hits)"}
    log(f"[bench] selection: {sel['ms']:.3f} ms, {n_tracks} tracks with {n_track_hits} hits")
    # full Kalman refit of the selected tracks (binary64)
    fits = tr.fits_output(tracks)
    tr.refit(hits, out, tracks, fits)
    torch.cuda.synchronize()
    s0.record(stream)
    for _ in range(5):
        tr.refit(hits, out, tracks, fits)
    s1.record(stream)
    torch.cuda.synchronize()
    fn = fits.numpy(n_tracks)
    ok = fn["flags"] == 1
    n_state, n_steps, n_upd = refit_work(batch, out, n_trk, tracks.numpy(n_tracks, n_track_hits), fn)
    refit_ms = s0.elapsed_time(s1) / 5
    refit_flops = REFIT_FLOPS_TRANSPORT * n_state + REFIT_FLOPS_STEP * n_steps + REFIT_FLOPS_UPDATE * n_upd
    refit = {"ms": refit_ms, "tracks": n_tracks, "done": int(ok.sum()),
             "chi2_per_ndf_mean": float(np.mean(fn["chi2"][ok] / np.maximum(fn["ndf"][ok], 1))) if ok.any() else None,
             "state_transports": n_state, "row_steps": n_steps, "updates": n_upd,
             "fp64_tflops": refit_flops / (refit_ms * 1e-3) / 1e12, "fp64_peak_tflops": PEAK_FP64_TFLOPS,
             "what": "full Kalman refit of the selected tracks: 5x5 covariance, coupled Jacobian, binary64"}
    log(f"[bench] refit: {refit['ms']:.3f} ms, {refit['done']} of {n_tracks} tracks, "
        f"chi2/ndf {refit['chi2_per_ndf_mean']}, {n_steps} row steps, {n_upd} updates, "
        f"{refit['fp64_tflops']:.2f} TFLOP/s binary64")
    # segment merging inside the sectors (after the refit)
    merge = merge_leg(tr, hits, out, tracks, fits, n_tracks, stream)
    log(f"[bench] merge: {merge['ms']:.3f} ms, {merge['links']} links among {n_tracks} tracks, "
        f"{merge['candidate_pairs']} pairs, {merge['transport_steps']} steps")
    del tracks, fits
    if not args.no_dead_band and args.workload == "batch64":
        import synth
        bd = synth.batch_workload(seed=args.seed, n_events=64, dead_rows=DEAD_BAND)
        hd = DeviceHits(bd.y, bd.z, bd.row, bd.hit_offset, dev)
        od = tr.output(hd)
        tr.track(hd, od)
        st_d, _ = tr.result()
        if st_d != C.CATPC_OK:
            raise SystemExit(f"catpc status {st_d}: {C.catpc_last_error()}")
        td = tr.tracks_output(hd, od)
        tr.select(hd, od, td)
        nt_d, _ = tr.select_result()
        fd = tr.fits_output(td)
        tr.refit(hd, od, td, fd)
        merge["dead_band"] = merge_leg(tr, hd, od, td, fd, nt_d, stream)
        merge["dead_band"]["rows"] = [DEAD_BAND[0], DEAD_BAND[0] + DEAD_BAND[1] - 1]
        merge["dead_band"]["hits"] = int(hd.n_hits)
        log(f"[bench] merge, dead rows {DEAD_BAND[0]}-{DEAD_BAND[0] + DEAD_BAND[1] - 1}: "
            f"{merge['dead_band']['ms']:.3f} ms, {merge['dead_band']['links']} links among {nt_d} tracks, "
            f"{merge['dead_band']['candidate_pairs']} pairs, {merge['dead_band']['transport_steps']} steps, "
            f"{merge['dead_band']['fp64_tflops']:.2f} TFLOP/s binary64")
        del bd, hd, od, td, fd
        tr.track(hits, out)  # leave the context's last call on the main workload
        tr.result()

    flops = (work[0] * FLOPS_PER_TRANSPORT + work[1] * FLOPS_PER_UPDATE + work[3] * FLOPS_PER_SEARCH +
             work[2] * FLOPS_PER_CANDIDATE)
    tc_ms = stages["tracklets"]
    nf_ms = stages["neighbours"]
    rl_tc = {"kernel": "k_tracklets", "bound": "alu", "achieved": flops / (tc_ms * 1e-3) / 1e12,
             "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "traffic": None, "launch_ms": tc_ms,
             "algorithmic_flops": float(flops), "work_counts": work.tolist()}
    rl_tc["frac"] = rl_tc["achieved"] / rl_tc["peak"]
    nf_bytes = NF_BYTES_PER_HIT * hits.n_hits
    # the neighbour stage: the LDS-staged kernel, or (nf_lds_kb = 0) the in-place one
    nf_kernel = "k_nf_flat" if tuning["nf_lds_kb"] == 0 else "k_neighbours"
    rl_nf = {"kernel": nf_kernel, "bound": "hbm", "achieved": nf_bytes / (nf_ms * 1e-3) / 1e9,
             "peak": HBM_PEAK_GBS, "unit": "GB/s", "traffic": None, "launch_ms": nf_ms,
             "algorithmic_bytes": nf_bytes}
    rl_nf["frac"] = rl_nf["achieved"] / rl_nf["peak"]
    others = {}
    for kern, stage, per_hit in (("k_grid", "grid", GRID_BYTES_PER_HIT), ("k_clean_start", "clean_start",
                                                                          CLEAN_BYTES_PER_HIT),
                                 ("k_row_index", "row_index", ROWIDX_BYTES_PER_HIT)):
        ms_k = stages[stage]
        byts = per_hit * hits.n_hits
        others[kern] = {"kernel": kern, "bound": "hbm", "achieved": byts / (ms_k * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "traffic": None, "launch_ms": ms_k, "algorithmic_bytes": byts}
        others[kern]["frac"] = others[kern]["achieved"] / HBM_PEAK_GBS
    traffic = profiled_traffic(args.workload, tuning)
    for rl in (rl_tc, rl_nf, *others.values()):
        parts = [traffic.get(kn) for kn in rl["kernel"].split("+")]
        if all(parts):
            f = sum(t["fetch_bytes"] for t in parts)
            wr = sum(t["write_bytes"] for t in parts)
            rl["traffic"] = f + wr
            rl["traffic_fetch"], rl["traffic_write"] = f, wr
            rl["traffic_source"] = os.path.relpath(TRAFFIC_PROFILE, ROOT)
    dominant = rl_tc if tc_ms >= nf_ms else rl_nf

    # plain form: the same stages launched sector by sector
    plain = None
    if args.plain_steps > 0:
        tr.track(hits, out, "plain")
        tr.result()
        torch.cuda.synchronize()
        pev = [torch.cuda.Event(enable_timing=True) for _ in range(args.plain_steps + 1)]
        pev[0].record(stream)
        for k in range(args.plain_steps):
            tr.track(hits, out, "plain")
            pev[k + 1].record(stream)
        torch.cuda.synchronize()
        st, n2 = tr.result()
        pms = float(np.median([pev[k].elapsed_time(pev[k + 1]) for k in range(args.plain_steps)]))
        plain = {"hits_per_s": hits.n_hits / (pms * 1e-3), "ms_per_step": pms, "steps": args.plain_steps,
                 "timing": "median of the HIP-event-timed steps", "launches_per_step": 8 * hits.n_sectors + 1,
                 "status": int(st), "n_tracklets": n2}
        log(f"[bench] plain: {pms:.3f} ms/step, {plain['hits_per_s']:.4g} hits/s")

    scheduling = None
    if not args.no_scheduling:
        scheduling = scheduling_leg(batch, tuning, hits.n_hits, log)
        scheduling["plain_1_queue"] = {"ms_per_step": plain["ms_per_step"], "hits_per_s": plain["hits_per_s"]} \
            if plain else None
        scheduling["batch_1_instance"] = {"ms_per_step": ms_step, "hits_per_s": value}
        scheduling["note"] = ("HIP maps a process's streams onto GPU_MAX_HW_QUEUES hardware queues (4 here, the "
                              "default), so the 8 streams of the 8-queue form share 4 hardware queues")

    serving = None
    if args.serve_events > 0:
        serving = serving_leg(args, tuning, log)

    peaks = None
    if not args.no_peaks:
        peaks = peak_probes(torch, C, dev, stream, log)
        for rl in (rl_tc, rl_nf):
            key = "fma_tflops" if rl["bound"] == "alu" else "copy_gbs"
            rl["achievable_peak"] = peaks[key]
            rl["frac_of_achievable"] = rl["achieved"] / peaks[key]

    precision, prec_keep = None, {}
    if not args.no_precision:
        precision, prec_keep = precision_leg(torch, tuning, log)

    configs = None
    if not args.no_configs:
        configs = config_lines(torch, tuning, args.seed, log)

    linearity = None
    if not args.no_linearity:
        linearity = linearity_leg(torch, tuning, args.seed, log)

    cpu = None
    if not args.no_cpu_baseline:
        cores = min(16, os.cpu_count() or 1)
        log(f"[bench] oracle on a sample, {cores} threads")
        cpu = cpu_baseline(batch, args.cpu_hits, cores)
        log(f"[bench] oracle: {cpu['value']:.4g} hits/s")
        one = cpu_baseline(batch, args.cpu_hits_1, 1)
        log(f"[bench] oracle, one thread: {one['value']:.4g} hits/s")
        cpu["single_thread"] = {"value": one["value"], "sample": one["sample"]}
        four = cpu_baseline(batch, args.cpu_hits_4, 4)
        log(f"[bench] oracle, four threads: {four['value']:.4g} hits/s")
        cpu["four_threads"] = {"value": four["value"], "sample": four["sample"]}
        cpu["gpu_over_four_threads"] = value / four["value"]
        # the same oracle leg, untimed: binary32 GPU parameters against the
        # binary64 oracle refit of their hits (config 3 and sampled sectors of
        # this batch, every k-th by size)
        checks = {}
        for (name, prec), (b1, t1, p1) in prec_keep.items():
            if (name, prec) in (("sector", 0), ("sector_precise_clusters", 1)):
                checks[f"{name}_precision_{prec}"] = parameter_check([(b1.y, b1.z, b1.row_x, t1, p1)])
        if args.workload == "batch64":
            sizes = np.diff(batch.hit_offset)
            pick = sorted(np.argsort(-sizes, kind="stable")[::16].tolist())
            off = out.tracklet_offset.cpu().numpy()
            items = []
            for sct in pick:
                a0, a1 = int(off[sct]), int(off[sct + 1])
                sec = batch.sector(sct)
                t1 = {"param": out.param[a0:a1].cpu().numpy(), "row_hit": out.row_hit[a0:a1].cpu().numpy(),
                      "start_row": out.start_row[a0:a1].cpu().numpy(), "flags": out.flags[a0:a1].cpu().numpy()}
                items.append((sec["y"], sec["z"], batch.row_x, t1, C.catpc_default_params()))
            checks[f"batch64_sample_{len(pick)}_sectors"] = parameter_check(items)
        for k, v in checks.items():
            log(f"[bench] parameters vs binary64 oracle, {k}: {v['fraction_strict']} of {v['tracklets']} strict")
        if precision is not None:
            precision["parameter_check"] = checks | {"computed_by": "the oracle leg (binary64 refit of the GPU "
                                                                   "tracklets' hits)"}
        cpu["paper_context"] = ("the paper quotes its GPU tracker at about 10x four CPU cores on its own Run-1 "
                                "hardware (Sec. 1); context only, different hardware, code and data")
        cpu["nproc"] = os.cpu_count()
        cpu["cpu_model"] = cpu_model()

    res = {"metric": METRIC, "value": value, "unit": "hits/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_step, "ms_per_step_median": float(np.median(step_ms)), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic (seeded helix events, no recorded data)",
           "config": {"workload": desc, "n_hits": hits.n_hits, "n_sectors": hits.n_sectors,
                      "n_tracklets": n_trk, "seed": args.seed, "form": "batched: fixed launch chain over all "
                      "sectors, persistent tracklet kernel, hipGraph replay", "parallelism": "single GPU",
                      "tuning": tuning, "tuning_source": tuning_src},
           "plain": plain, "batched_over_plain": (value / plain["hits_per_s"]) if plain else None,
           "serving": serving, "stages_ms": stages, "roofline": {k: v for k, v in dominant.items() if k != "kernel"} |
           {"kernel": dominant["kernel"]}, "rooflines": {"k_tracklets": rl_tc, "neighbours": rl_nf, **others},
           "selection": sel, "refit": refit, "merge": merge, "scheduling": scheduling, "achievable_peaks": peaks, "precision": precision, "configs": configs, "linearity": linearity, "cpu_baseline": cpu}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
