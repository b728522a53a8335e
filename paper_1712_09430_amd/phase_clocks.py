"""Where the row-synchronous tracklet kernel's time goes, phase by phase, on
the batch64 workload (64 events, seed 1) with the cached launch shape.

Loads the profiling build of the library (`libcatpc_phase.so`, built by
`build.build_phase_clocks()` or `__graft_entry__.build()`), whose kernel sums
shader-clock cycles per phase over its waves (`catpc_phase_clocks`), runs the
batched chain once to warm up and once measured, and prints a Markdown table:
cycles per slot batch of each phase (start of the batch; outward pass = seed
chain and outward following; record store and back-transport; inward pass),
row steps and cycles per row step of the two passes, and the tracklet stage
time of the profiling build next to the product build's.

    python -m paper_1712_09430_amd.phase_clocks
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def stage_ms(tracker, hits, out, reps=5):
    import numpy as np
    from . import catpc as C
    s = np.median(np.stack([tracker.stage_times(hits, out) for _ in range(reps)]), axis=0)
    return float(s[C.STAGES.index("tracklets")])


def main():
    import numpy as np
    import torch

    import synth
    from . import autotune, build, catpc as C
    from .tracker import DeviceHits, Tracker

    if not os.path.exists(build.PHASE_LIB):
        raise SystemExit(f"profiling build missing: {build.PHASE_LIB} (run __graft_entry__.build())")
    b = synth.batch_workload(seed=1)
    tuning = autotune.cached_tuning()
    hits = DeviceHits(b.y, b.z, b.row, b.hit_offset, "cuda:0")
    # product build first, then the profiling build in a fresh handle
    tr = Tracker(b.row_x, hits.n_hits, hits.n_sectors, tuning=tuning, device="cuda:0")
    out = tr.output(hits)
    tr.track(hits, out)
    tr.result()
    product_ms = stage_ms(tr, hits, out)
    tr.close()
    C.use_library(build.PHASE_LIB)
    tr = Tracker(b.row_x, hits.n_hits, hits.n_sectors, tuning=tuning, device="cuda:0")
    out = tr.output(hits)
    tr.track(hits, out)
    tr.result()
    torch.cuda.synchronize()
    C.catpc_phase_clocks(clear=True)
    tr.track(hits, out)
    st, n = tr.result()
    torch.cuda.synchronize()
    if st != C.CATPC_OK:
        raise SystemExit(f"catpc status {st}: {C.catpc_last_error()}")
    g = np.array(C.catpc_phase_clocks(), dtype=np.float64)
    profiled_ms = stage_ms(tr, hits, out)
    tr.close()
    nb, nw = g[6], g[8]
    phases = [("start of a slot batch (slots, chain records, seed state)", g[0], None),
              ("outward pass (seed chain and outward following)", g[1], g[4]),
              ("record store and back-transport to the start row", g[2], None),
              ("inward pass (inward following)", g[3], g[5])]
    total = sum(p[1] for p in phases)
    print("| phase | cycles per slot batch | share % | row steps per batch | cycles per row step |")
    print("|---|---:|---:|---:|---:|")
    for name, cyc, steps in phases:
        cols = [f"{cyc / nb:.0f}", f"{100 * cyc / total:.1f}",
                f"{steps / nb:.1f}" if steps is not None else "",
                f"{cyc / steps:.0f}" if steps else ""]
        print(f"| {name} | " + " | ".join(cols) + " |")
    print()
    print(f"waves {nw:.0f}, slot batches {nb:.0f} ({nb / nw:.2f} per wave), {n} tracklets; "
          f"whole-wave cycles {g[7] / nw:.0f} per wave")
    print(f"tracklet stage: product build {product_ms:.4f} ms, profiling build {profiled_ms:.4f} ms")


if __name__ == "__main__":
    main()
