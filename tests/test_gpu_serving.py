"""Serving form: continuous batching of an event stream.  Each event's result
is the same alone and in the mix (bit for bit: all indices are sector-local
and sectors are independent), whatever batch and slot it landed in."""
import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection: the first import on a fresh box is slow)

import synth

pytestmark = pytest.mark.gpu


def test_results_alone_equal_results_in_the_mix():
    from paper_1712_09430_amd import serve
    pool = synth.event_pool(seed=5, n_events=6, lo=20, hi=2000)
    rng = np.random.default_rng(1)
    order = rng.integers(0, len(pool), 40)
    # fast arrivals: batches of several events, several slots in flight
    arrival = serve.poisson_arrivals(len(order), 5000.0, seed=2)
    src = serve.EventStream(pool, order, arrival, pool[0].row_x)
    mix = serve.serve(src, n_slots=3, slot_hits=1_500_000, slot_sectors=36 * 8, keep_results=True,
                      keep_rows=True, out_frac=0.001)
    assert mix["batches"] < len(order)  # events were batched together
    assert np.all(np.isfinite(mix["latency_s"])) and np.all(mix["latency_s"] > 0)
    for p in range(len(pool)):
        alone_src = serve.EventStream(pool, [p], [0.0], pool[0].row_x)
        alone = serve.serve(alone_src, n_slots=1, slot_hits=1_500_000, slot_sectors=36 * 8, keep_results=True,
                            keep_rows=True)["results"][0]
        for e in np.flatnonzero(order == p):
            got = mix["results"][e]
            assert np.array_equal(got["toff"], alone["toff"])
            assert np.array_equal(got["rows"], alone["rows"])
            for f, v in alone["trk"].items():
                assert np.array_equal(got["trk"][f].view(np.uint8), v.view(np.uint8)), f


def test_hbm_budget_limits_the_slots():
    from paper_1712_09430_amd import serve
    pool = synth.event_pool(seed=6, n_events=3, lo=20, hi=300)
    src = serve.EventStream(pool, [0, 1, 2, 0, 1, 2], serve.poisson_arrivals(6, 2000.0, seed=3), pool[0].row_x)
    with pytest.raises(ValueError):
        serve.serve(src, n_slots=4, slot_hits=200_000, slot_sectors=36 * 4, hbm_budget=1)


def test_small_budget_runs_with_one_slot():
    from paper_1712_09430_amd import serve
    pool = synth.event_pool(seed=6, n_events=3, lo=20, hi=300)
    src = serve.EventStream(pool, [0, 1, 2, 0, 1, 2], serve.poisson_arrivals(6, 2000.0, seed=3), pool[0].row_x)
    probe = serve.Slot(pool[0].row_x, 200_000, 36 * 4, None, None, "cuda:0", 0.01, False)
    fp = probe.footprint()
    probe.tracker.close()
    res = serve.serve(src, n_slots=4, slot_hits=200_000, slot_sectors=36 * 4, hbm_budget=int(1.5 * fp))
    assert res["slots"] == 1 and res["n_events"] == 6
