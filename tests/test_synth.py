"""The seeded input generator: published RNG vectors and the structure of the
synthetic events (row-sorted sectors, hits on the pad-row planes, acceptance)."""
import math
import os

import numpy as np

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) if l.strip() and l[0] != "#"]
    assert len(rows) == 3
    for r in rows:
        v = [int(w, 16) for w in r]
        assert synth.philox4x32_10(v[0:4], v[4:6]).tolist() == v[6:10]


def test_row_positions():
    rx = synth.row_x()
    assert rx.dtype == np.float32 and len(rx) == 159
    assert rx[0] == np.float32(85.0) and rx[-1] == np.float32(247.0)
    assert np.all(np.diff(rx) > 0)
    np.testing.assert_allclose(np.diff(rx.astype(np.float64)), 162.0 / 158.0, atol=2 * 2.0 ** -16)


def test_sector_event_structure():
    b = synth.sector_workload(seed=0, truth=True)
    assert b.n_sectors == 1
    s = b.sector(0)
    assert np.all(np.diff(s["row"]) >= 0)
    assert np.array_equal(s["x"], b.row_x[s["row"]])
    sig = s["label"] >= 0
    # signal: one hit per (track, row)
    key = s["label"][sig].astype(np.int64) * 1000 + s["row"][sig]
    assert len(np.unique(key)) == sig.sum()
    # unsmeared positions inside the sector acceptance, z on side A
    xr = b.row_x[s["row"]].astype(np.float64)
    assert np.all(np.abs(s["y_true"][sig]) <= xr[sig] * math.tan(math.radians(10)) + 1e-9)
    assert np.all(s["z_true"][sig] >= 0) and np.all(s["z_true"][sig] <= 250)
    # smear ~ 0.1 cm
    dy = s["y"][sig] - s["y_true"][sig]
    assert abs(dy.std() - 0.1) < 0.01 and abs(dy.mean()) < 0.01
    # 10 % noise
    assert abs((~sig).sum() - round(0.1 * sig.sum())) <= 1


def test_hits_lie_on_the_closed_form_helix():
    b = synth.sector_workload(seed=2, truth=True, sigma=0.0, noise_frac=0.0)
    s = b.sector(0)
    tr = b.tracks[0]
    for i in range(0, len(s["y"]), 97):
        t = s["label"][i]
        qpt = tr["q"][t] / tr["pt"][t]
        # find the path length at which the helix reaches this row plane
        lo, hi = 0.0, 400.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if synth.helix_point(qpt, math.sinh(tr["eta"][t]), tr["phi0"][t], b.bz, s["alpha"], mid)[0] < s["x"][i]:
                lo = mid
            else:
                hi = mid
        p = synth.helix_point(qpt, math.sinh(tr["eta"][t]), tr["phi0"][t], b.bz, s["alpha"], lo)
        assert abs(p[1] - s["y_true"][i]) < 1e-7 and abs(p[2] - s["z_true"][i]) < 1e-7
        assert abs(p[3] - s["sinphi_true"][i]) < 1e-9


def test_event_and_batch_shapes():
    e = synth.event_workload(seed=3, n_tracks=500)
    assert e.n_sectors == 36
    for s in range(36):
        r = e.row[e.hit_offset[s]:e.hit_offset[s + 1]]
        assert np.all(np.diff(r) >= 0)
    z = e.z
    for s in range(36):
        zz = z[e.hit_offset[s]:e.hit_offset[s + 1]]
        if len(zz):
            assert (np.median(zz) > 0) == (s < 18)
    m = synth.multiplicities(1, 64)
    assert min(m) >= 20 and max(m) < 10000 and len(m) == 64


def test_determinism():
    a = synth.sector_workload(seed=7)
    b = synth.sector_workload(seed=7)
    c = synth.sector_workload(seed=8)
    assert np.array_equal(a.y, b.y) and np.array_equal(a.row, b.row)
    assert a.n_hits != c.n_hits or not np.array_equal(a.y, c.y)


def test_workloads_keep_the_row_count_they_are_given():
    """Every workload helper builds its row planes for the n_rows the events
    were generated with (the row values stay below it)."""
    import synth
    for b in (synth.sector_workload(seed=1, n_tracks=20, n_rows=64),
              synth.tracks_workload({"q": [1], "pt": [1.0], "eta": [0.2], "phi0": [synth.sector_alpha(0)]},
                                    n_rows=30, sigma=0.0, noise_frac=0.0),
              synth.event_workload(seed=1, n_tracks=30, n_rows=17),
              synth.batch_workload(seed=1, n_events=2, n_rows=40),
              synth.event_pool(seed=1, n_events=2, n_rows=25)[1]):
        n = len(b.row_x)
        assert n == b.n_rows and int(b.row.max()) < n and n in (64, 30, 17, 40, 25)
        assert np.all(np.diff(b.row_x) > 0)
