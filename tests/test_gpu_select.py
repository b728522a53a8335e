"""Tracklet selection on the GPU against the oracle (Sec. 2 item 2): per
sector the selected tracks (their tracklet, their hits in row order) equal the
oracle's selection of the oracle's own tracklets, bit for bit; at full size on
sampled sectors plus properties over all sectors; edge cases and capacity
reports."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection: the first import on a fresh box is slow)

import oracle
import synth
from _harness import oracle_params, run_gpu

pytestmark = pytest.mark.gpu


def select_gpu(tr, hits, out, tracks=None):
    if tracks is None:
        tracks = tr.tracks_output(hits, out)
    tr.select(hits, out, tracks)
    nt, nh = tr.select_result()
    return tracks, tracks.numpy(nt, nh), nt, nh


def compare_select(batch, s, g, params):
    """Mismatches between the GPU selection of sector s and the oracle's."""
    sec = batch.sector(s)
    P = oracle_params(params)
    o = oracle.track_sector(sec["y"], sec["z"], sec["row"], batch.row_x, P, "f32")
    _, want = oracle.select(len(sec["y"]), o["row_hit"], o["n_hits"], o["flags"], P.min_hits)
    k0, k1 = int(g["track_offset"][s]), int(g["track_offset"][s + 1])
    got = []
    for k in range(k0, k1):
        h0 = int(g["track_hit_offset"][k])
        got.append((int(g["track_tracklet"][k]), g["track_hits"][h0:h0 + int(g["track_n_hits"][k])]))
    if len(got) != len(want):
        return [f"sector {s}: {len(got)} tracks, oracle {len(want)}"]
    bad = []
    for (tg, hg), (tw, hw) in zip(got, want):
        if tg != tw or not np.array_equal(hg, hw):
            bad.append(f"sector {s}: track of tracklet {tg} (oracle {tw}) differs")
    return bad


def check_all(batch, g, params, sectors):
    with ThreadPoolExecutor(max_workers=8) as ex:
        bad = [m for r in ex.map(lambda s: compare_select(batch, s, g, params), sectors) for m in r]
    assert not bad, "\n".join(bad[:20])


@pytest.mark.parametrize("seed", [1, 2])
def test_one_sector_matches_oracle(seed):
    from paper_1712_09430_amd import catpc as C
    b = synth.sector_workload(seed=seed, n_tracks=300)
    tr, hits, out, st, n = run_gpu(b)
    _, g, nt, nh = select_gpu(tr, hits, out)
    assert nt > 0 and nh >= nt * 10
    check_all(b, g, C.catpc_default_params(), [0])


def test_dense_row_chunks_claim_in_memory():
    """A sector dense enough that most chunks of 16 rows hold more hits than
    the claim keeps in LDS (8192): those chunks claim on the owner words in
    memory, the last one in LDS; the selection still equals the oracle's."""
    from paper_1712_09430_amd import catpc as C
    b = synth.sector_workload(seed=5, n_tracks=900)
    per_row = np.bincount(b.row, minlength=len(b.row_x))
    chunks = [int(per_row[r:r + 16].sum()) for r in range(0, len(b.row_x), 16)]
    assert max(chunks) > 8192 and min(chunks) <= 8192
    tr, hits, out, st, n = run_gpu(b)
    assert st == C.CATPC_OK
    _, g, nt, nh = select_gpu(tr, hits, out)
    assert nt > 300
    check_all(b, g, C.catpc_default_params(), [0])


def test_uneven_batch_graph_and_plain_launches_agree():
    from paper_1712_09430_amd import catpc as C
    b = synth.batch_workload(seed=7, n_events=3, lo=20, hi=3000)
    for use_graph in (1, 0):
        tr, hits, out, st, n = run_gpu(b, tuning={"use_graph": use_graph})
        tracks, g, nt, nh = select_gpu(tr, hits, out)
        check_all(b, g, C.catpc_default_params(), range(b.n_sectors))
        # a second selection (graph replay) on cleared buffers gives the same tracks
        tracks.track_hits.fill_(-5)
        tracks.track_tracklet.fill_(-5)
        _, g2, nt2, nh2 = select_gpu(tr, hits, out, tracks)
        assert (nt2, nh2) == (nt, nh)
        for k in g:
            assert np.array_equal(g[k], g2[k]), k


def test_full_batch_sampled_sectors_and_properties():
    from paper_1712_09430_amd import autotune
    from paper_1712_09430_amd import catpc as C
    b = synth.batch_workload(seed=1, n_events=64)
    cached = autotune.cached_tuning()
    tr, hits, out, st, n = run_gpu(b, tuning=cached)
    assert st == C.CATPC_OK
    tracks, g, nt, nh = select_gpu(tr, hits, out)
    sizes = np.diff(b.hit_offset)
    order = np.argsort(sizes, kind="stable")
    rng = np.random.default_rng(99)
    sample = sorted(set(order[-4:].tolist()) | set(rng.choice(b.n_sectors, 16, replace=False).tolist()))
    check_all(b, g, C.catpc_default_params(), sample)
    # properties over every sector
    toff = g["track_offset"]
    assert toff[0] == 0 and toff[-1] == nt and np.all(np.diff(toff) >= 0)
    assert np.all(g["track_n_hits"] >= 10)
    assert np.array_equal(g["track_hit_offset"], np.concatenate([[0], np.cumsum(g["track_n_hits"])[:-1]]))
    sec_of_track = np.repeat(np.arange(b.n_sectors), np.diff(toff))
    glob = b.hit_offset[np.repeat(sec_of_track, g["track_n_hits"])] + g["track_hits"]
    assert len(np.unique(glob)) == nh  # no hit in two tracks
    rows = b.row[glob]
    same = np.repeat(np.arange(nt), g["track_n_hits"])
    step = np.diff(rows)[np.diff(same) == 0]
    assert np.all(step > 0)  # rows ascending within a track


def test_capacity_and_state_reports():
    from paper_1712_09430_amd import catpc as C
    from paper_1712_09430_amd.tracker import DeviceTracks
    b = synth.sector_workload(seed=3, n_tracks=200)
    tr, hits, out, st, n = run_gpu(b)
    _, g, nt, nh = select_gpu(tr, hits, out)
    small = DeviceTracks(hits.n_sectors, max(nt - 1, 0), nh, "cuda:0")
    tr.select(hits, out, small)
    with pytest.raises(C.CatpcError) as e:
        tr.select_result()
    assert e.value.status == C.CATPC_E_CAPACITY
    # tracklet output holding only part of the tracklets
    tr2, hits2, out2, st2, n2 = run_gpu(b, capacity=max(n // 2, 1))
    assert st2 == C.CATPC_E_CAPACITY
    tr2.select(hits2, out2, tr2.tracks_output(hits2, out2))
    with pytest.raises(C.CatpcError) as e:
        tr2.select_result()
    assert e.value.status == C.CATPC_E_CAPACITY
    # a new track call invalidates the selection
    tr.track(hits, out)
    tr.result()
    with pytest.raises(C.CatpcError) as e:
        tr.select_result()
    assert e.value.status == C.CATPC_E_STATE


def test_record_entries_outside_their_row_are_reported():
    """A record entry that names a hit of another row, or no hit of the
    sector, is skipped and reported as CATPC_E_INVALID; after a new track call
    the selection equals the oracle's again."""
    from paper_1712_09430_amd import catpc as C
    b = synth.sector_workload(seed=4, n_tracks=200)
    tr, hits, out, st, n = run_gpu(b)
    t = out.tracklets_numpy(n)
    v = int(np.flatnonzero(t["flags"] & 1)[0])  # a valid tracklet
    rows = np.flatnonzero(t["row_hit"][v] >= 0)
    r_a, r_b = int(rows[0]), int(rows[1])  # two rows of one chunk of 16 rows, as a rule
    for bad in (int(t["row_hit"][v][r_b]), hits.n_hits + 5):
        out.row_hit[v, r_a] = bad
        tr.select(hits, out, tr.tracks_output(hits, out))
        with pytest.raises(C.CatpcError) as e:
            tr.select_result()
        assert e.value.status == C.CATPC_E_INVALID
    tr.track(hits, out)
    tr.result()
    _, g, nt, nh = select_gpu(tr, hits, out)
    check_all(b, g, C.catpc_default_params(), [0])


def test_empty_inputs():
    from paper_1712_09430_amd import catpc as C
    from paper_1712_09430_amd.tracker import DeviceHits, Tracker
    tr = Tracker(synth.row_x(), 10, 4)
    hits = DeviceHits(np.zeros(0), np.zeros(0), np.zeros(0), np.array([0, 0, 0]))
    out = tr.output(hits, 1)
    tr.track(hits, out)
    st, n = tr.result()
    assert st == C.CATPC_OK and n == 0
    _, g, nt, nh = select_gpu(tr, hits, out)
    assert (nt, nh) == (0, 0) and g["track_offset"].tolist() == [0, 0, 0]
