"""The no-allocation entry point (catpc_track_batch_noalloc) against the
batched form with a context (catpc_track_batch) on the same inputs, through
the C ABI: every link and tracklet field bit for bit, on two calls in a row
(the second with a smaller input, so it runs on what the first left in the
fixed workspace).  Collected last: it shares the device array with nothing
else, and a failure here hides no other test."""
import numpy as np
import pytest
import torch  # noqa: F401

import synth
from _harness import TRACKLET_KEYS, run_gpu

pytestmark = pytest.mark.gpu


def _noalloc(b, tuning=None):
    import torch
    from paper_1712_09430_amd import catpc as C
    from paper_1712_09430_amd.tracker import DeviceHits, DeviceOutput
    hits = DeviceHits(b.y, b.z, b.row, b.hit_offset, "cuda:0")
    rx = torch.from_numpy(np.ascontiguousarray(b.row_x, np.float32)).cuda()
    out = DeviceOutput(hits.n_hits, hits.n_sectors, hits.n_hits // 3 + 1, len(b.row_x), "cuda:0")
    status = torch.full((1,), -1, dtype=torch.int64, device="cuda:0")
    stream = torch.cuda.current_stream()
    C.catpc_track_batch_noalloc(len(b.row_x), rx.data_ptr(), C.catpc_default_params(), tuning, hits.struct,
                                out.struct, status.data_ptr(), stream.cuda_stream)
    torch.cuda.synchronize()
    n = int(out.tracklet_offset[-1].item()) if hits.n_sectors > 0 else 0
    return out, int(status.item()), n


def _same(b, tuning=None):
    from paper_1712_09430_amd import catpc as C
    _, _, ref, st, n0 = run_gpu(b)
    assert st == C.CATPC_OK
    out, status, n = _noalloc(b, tuning)
    assert status == 0 and n == n0
    l0, l1 = ref.links_numpy(), out.links_numpy()
    for k in l0:
        assert np.array_equal(l0[k], l1[k]), k
    t0, t1 = ref.tracklets_numpy(n0), out.tracklets_numpy(n)
    for k in TRACKLET_KEYS:
        a, c = t0[k], t1[k]
        assert np.array_equal(a.view(np.uint8) if a.dtype == np.float32 else a,
                              c.view(np.uint8) if c.dtype == np.float32 else c), k
    return n


def test_no_alloc_entry_point_matches_the_batched_form_twice():
    big = synth.batch_workload(seed=31, n_events=2, lo=500, hi=3000)
    small = synth.sector_workload(seed=32)
    assert small.n_hits < big.n_hits
    n1 = _same(big)
    n2 = _same(small)
    assert n1 > n2 > 0
