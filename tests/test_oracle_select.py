"""Pins for the tracklet-selection oracle (Sec. 2 item 2: duplicate
tracklets grown from several seeds of one segment reduce to one).
Hand-built cases decide every rule of the reading (weight = hit count, ties
to the smaller tracklet, invalid tracklets take no part, a tracklet needs
min_hits hits of its own, dropped tracklets hand nothing on); properties hold
on full sectors."""
import math

import numpy as np

import oracle
import synth

R = 20


def rec(*rows_hits):
    """One tracklet record over R rows from (row, hit) pairs."""
    r = np.full(R, -1, np.int32)
    for row, h in rows_hits:
        r[row] = h
    return r


def run(records, flags=None, min_hits=3, n_hits=100):
    rh = np.stack(records).astype(np.int32)
    n = (rh >= 0).sum(1).astype(np.int32)
    fl = np.ones(len(records), np.int32) if flags is None else np.asarray(flags, np.int32)
    return oracle.select(n_hits, rh, n, fl, min_hits=min_hits)


def test_longer_tracklet_takes_shared_hits():
    a = rec(*[(r, r) for r in range(0, 8)])          # 8 hits
    b = rec(*[(r, r) for r in range(5, 8)], *[(r, 50 + r) for r in range(8, 12)])  # 7 hits, 3 shared
    owned, tracks = run([b, a])
    assert owned.tolist() == [4, 8]
    assert [t for t, _ in tracks] == [0, 1]
    assert tracks[0][1].tolist() == [58, 59, 60, 61]   # b keeps its own hits, rows ascending
    assert tracks[1][1].tolist() == list(range(8))


def test_equal_counts_go_to_the_smaller_tracklet():
    a = rec(*[(r, r) for r in range(0, 6)])
    b = rec(*[(r, r) for r in range(3, 9)])          # 6 hits, rows 3-5 shared
    owned, tracks = run([a, b])
    assert owned.tolist() == [6, 3]
    owned, tracks = run([b, a])                      # swapped: the index decides, not the hits
    assert owned.tolist() == [6, 3]


def test_a_tracklet_below_min_hits_after_sharing_is_dropped():
    a = rec(*[(r, r) for r in range(0, 10)])
    b = rec(*[(r, r) for r in range(6, 10)], (10, 70), (11, 71))   # 6 hits, keeps 2
    owned, tracks = run([a, b], min_hits=3)
    assert owned.tolist() == [10, 0] and len(tracks) == 1


def test_invalid_tracklets_take_no_part():
    a = rec(*[(r, r) for r in range(0, 12)])         # longest, but not valid
    b = rec(*[(r, r) for r in range(0, 5)])
    owned, tracks = run([a, b], flags=[0, 1])
    assert owned.tolist() == [0, 5]


def test_dropped_tracklets_hand_nothing_on():
    best = rec(*[(r, r) for r in range(0, 15)])                           # 15 hits
    mid = rec(*[(r, r) for r in range(9, 15)], *[(r, 30 + r) for r in range(15, 19)])   # 10: keeps 4
    low = rec(*[(r, 30 + r) for r in range(15, 18)], (18, 80), (19, 81))                # 5: loses 3 to mid
    owned, tracks = run([best, mid, low], min_hits=5)
    # mid is dropped (4 < 5), and the hits it took from low are not handed back
    assert owned.tolist() == [15, 0, 0]


def test_empty_and_no_valid():
    owned, tracks = oracle.select(10, np.zeros((0, R), np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert len(owned) == 0 and tracks == []
    owned, tracks = run([rec((0, 1), (1, 2), (2, 3))], flags=[0])
    assert owned.tolist() == [0] and tracks == []


def test_properties_on_full_sectors():
    P = oracle.Params()
    for seed in (1, 2, 3):
        b = synth.sector_workload(seed=seed, n_tracks=300)
        s = b.sector(0)
        o = oracle.track_sector(s["y"], s["z"], s["row"], b.row_x, P, "f32")
        owned, tracks = oracle.select(len(s["y"]), o["row_hit"], o["n_hits"], o["flags"], P.min_hits)
        seen = np.zeros(len(s["y"]), bool)
        for t, hits in tracks:
            assert o["flags"][t] & oracle.VALID
            assert len(hits) == owned[t] >= P.min_hits
            mine = o["row_hit"][t]
            assert set(hits.tolist()) <= set(mine[mine >= 0].tolist())
            assert np.all(np.diff(s["row"][hits]) > 0)        # one hit per row, rows ascending
            assert not seen[hits].any()                        # no hit in two selected tracks
            seen[hits] = True
        # a valid tracklet none of whose hits is shared with a heavier one is kept whole
        for t in np.flatnonzero(o["flags"] & oracle.VALID):
            mine = o["row_hit"][t]
            mine = set(mine[mine >= 0].tolist())
            heavier = [u for u in np.flatnonzero(o["flags"] & oracle.VALID)
                       if (o["n_hits"][u], -u) > (o["n_hits"][t], -t)]
            if all(not (mine & set(o["row_hit"][u][o["row_hit"][u] >= 0].tolist())) for u in heavier):
                assert owned[t] == len(mine)


def test_noise_free_tracks_give_one_segment_each():
    tracks = {"q": [1, -1, 1, -1], "pt": [6.0, 2.0, 1.0, 0.6], "eta": [0.1, 0.3, 0.5, 0.7],
              "phi0": [math.radians(a) for a in (4.0, 8.0, 12.0, 16.0)]}
    b = synth.tracks_workload(tracks, sigma=0.0, noise_frac=0.0)
    s = b.sector(0)
    P = oracle.Params()
    o = oracle.track_sector(s["y"], s["z"], s["row"], b.row_x, P, "f32")
    owned, sel = oracle.select(len(s["y"]), o["row_hit"], o["n_hits"], o["flags"], P.min_hits)
    lab = s["label"]
    got = sorted(int(lab[h[0]]) for _, h in sel)
    want = sorted(L for L in range(4) if (lab == L).sum() >= P.min_hits)
    assert got == want
    for _, h in sel:
        assert len(set(lab[h].tolist())) == 1 and len(h) == (lab == lab[h[0]]).sum()
