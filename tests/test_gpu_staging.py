"""The row-synchronous tracklet kernel copies the pad row its searching lanes
need into LDS, for the sector of the wave's first searching lane, when the
copy fits (rows of up to about 290 hits); other lanes and larger rows search
the grid in place.  Both paths, and waves that span many sectors, must give
the oracle's result bit for bit (Sec. 2 item 2: the closest cluster per row
inside the gate)."""
import math

import numpy as np
import pytest

import synth
from _harness import compare_sector, gpu_sector, run_gpu
from test_gpu_edges import A0, HandBatch, track_hits

pytestmark = pytest.mark.gpu

RX = synth.row_x()


def dense_rows_sector(seed=11):
    """Twelve tracks, and noise rows of 200 hits (the copy fits), 300 (about
    the limit) and 450 hits (16 bytes per hit alone exceed the copy), half of
    each near the tracks so that the gates hold many candidates."""
    rng = np.random.default_rng(seed)
    h = []
    for k in range(12):
        h += track_hits(1 if k % 2 else -1, 1.0 + 0.4 * k, 0.02 + 0.07 * k, A0 + math.radians(-5.5 + k))
    tracks = {}
    for r, y, z in h:
        tracks.setdefault(r, []).append((y, z))
    for r, n in ((40, 200), (80, 300), (120, 450)):
        x = float(RX[r])
        w = x * math.tan(math.radians(10.0))
        for i in range(n):
            if i % 2 and tracks.get(r):
                y0, z0 = tracks[r][i % len(tracks[r])]
                h.append((r, float(np.float32(y0 + rng.uniform(-2.0, 2.0))), float(np.float32(z0 + rng.uniform(-2.0, 2.0)))))
            else:
                h.append((r, float(np.float32(rng.uniform(-w, w))), float(np.float32(rng.uniform(-120.0, 120.0)))))
    return h


def small_sectors(n=150):
    """One track per sector (all on the sectors' z > 0 side, as sector 0 of
    the generator is): every wave of tracklets spans many sectors."""
    out = []
    for k in range(n):
        out.append(track_hits(1 if k % 3 else -1, 1.0 + 0.03 * k, 0.02 + 0.01 * (k % 50),
                              A0 + math.radians(-5.0 + 0.066 * k)))
    return out


TUNINGS = [
    {"tc_sync": 1, "bin_hits": 0.5},
    {"tc_sync": 1, "bin_hits": 4.0, "tc_block": 64},
    {"tc_sync": 0},
]


@pytest.mark.parametrize("k", range(len(TUNINGS)))
def test_dense_rows_and_many_sectors_match_the_oracle(k):
    from paper_1712_09430_amd import catpc as C
    b = HandBatch([dense_rows_sector()] + small_sectors())
    p = C.catpc_default_params()
    tr, hits, out, st, n = run_gpu(b, p, tuning=TUNINGS[k])
    assert st == C.CATPC_OK, C.catpc_last_error()
    links, trk = out.links_numpy(), out.tracklets_numpy(n)
    bad = []
    for s in range(b.n_sectors):
        bad += compare_sector(b, s, gpu_sector(b, out, links, trk, s), p)
    assert not bad, "\n".join(bad[:20])
    # the dense rows were searched: tracklets of the dense sector reach them
    g = gpu_sector(b, out, links, trk, 0)
    for r in (40, 80, 120):
        assert (g["row_hit"][:, r] >= 0).sum() >= 10, r
    # waves spanned sectors: most small sectors hold a tracklet
    per_sector = np.diff(links["tracklet_offset"])[1:]
    assert (per_sector > 0).mean() > 0.9
