"""The profiling build of the library (the tracklet kernel's phase clocks
compiled in, `paper_1712_09430_amd/libcatpc_phase.so`) computes what the
product build computes, bit for bit, and its counters are consistent with the
work: one count per slot batch (up to 64 slots of one sector), one per wave of
the persistent grid, row steps in both passes and cycles in every phase."""
import math

import numpy as np
import pytest

import synth
from _harness import TRACKLET_KEYS, run_gpu


@pytest.mark.gpu
def test_profiling_build_matches_the_product_build():
    import paper_1712_09430_amd.build as B
    from paper_1712_09430_amd import catpc as C
    from paper_1712_09430_amd.tracker import DeviceHits, Tracker
    b = synth.batch_workload(seed=5, n_events=3)
    tun = {"tc_sync": 1, "tc_block": 128, "tc_waves_per_cu": 8}
    tr, hits, out, st, n = run_gpu(b, tuning=tun)
    assert st == C.CATPC_OK, C.catpc_last_error()
    ref_links, ref = out.links_numpy(), out.tracklets_numpy(n)
    tr.close()
    tr2 = None
    try:
        C.use_library(B.PHASE_LIB)
        hits2 = DeviceHits(b.y, b.z, b.row, b.hit_offset, "cuda:0")
        tr2 = Tracker(b.row_x, hits2.n_hits, hits2.n_sectors, tuning=tun, device="cuda:0")
        out2 = tr2.output(hits2)
        C.catpc_phase_clocks(clear=True)
        tr2.track(hits2, out2)
        st2, n2 = tr2.result()
        assert st2 == C.CATPC_OK and n2 == n
        g = C.catpc_phase_clocks()
        links, trk = out2.links_numpy(), out2.tracklets_numpy(n2)
        for k in ref_links:
            assert np.array_equal(ref_links[k], links[k]), k
        for k in TRACKLET_KEYS:
            assert np.array_equal(ref[k].view(np.uint8), trk[k].view(np.uint8)), k
        per_sector = np.diff(ref_links["tracklet_offset"])
        batches = int(sum(math.ceil(int(c) / 64) for c in per_sector))
        start, outward, back, inward, out_steps, in_steps, nb, wave_cycles, waves = g
        assert nb == batches
        assert waves > 0 and waves % (tun["tc_block"] // 64) == 0
        assert out_steps > 0 and in_steps > 0
        assert min(start, outward, back, inward) > 0
        # every batch runs inside one wave's lifetime
        assert wave_cycles >= start + outward + back + inward
    finally:
        if tr2 is not None:
            tr2.close()
        C.use_library(B.LIB)
