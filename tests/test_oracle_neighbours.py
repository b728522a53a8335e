"""Pins for the oracle's neighbour finding (Sec. 2 item 1, Fig. 2c): hand-built
cases whose answer follows from the geometry, not from the oracle's formula."""
import math

import numpy as np
import pytest

import oracle
import synth

P = oracle.Params()


def sector(hits, row_x):
    """hits: list of (row, y, z) in the order given; returns row-sorted arrays
    and the permutation new index -> position in `hits`."""
    order = sorted(range(len(hits)), key=lambda i: (hits[i][0], i))
    row = np.array([hits[i][0] for i in order], np.int32)
    y = np.array([hits[i][1] for i in order], np.float32)
    z = np.array([hits[i][2] for i in order], np.float32)
    return y, z, row, order


RX = synth.row_x()


@pytest.mark.parametrize("mode", ["f32", "f64"])
def test_collinear_triplet_is_linked(mode):
    a, b = 0.08, 0.4  # y/x and z/x of a ray from the origin
    hits = [(r, RX[r] * a, RX[r] * b) for r in (40, 41, 42)]
    y, z, row, order = sector(hits, RX)
    up, dn = oracle.neighbours(y, z, row, RX, P, mode)
    # only the middle hit has both neighbours; rows 40 and 42 have none in 39 / 43
    assert up.tolist() == [-1, 2, -1] and dn.tolist() == [-1, 0, -1]


def test_first_and_last_row_get_no_links():
    hits = [(r, RX[r] * 0.05, RX[r] * 0.2) for r in (0, 1, 2, 156, 157, 158)]
    y, z, row, _ = sector(hits, RX)
    up, dn = oracle.neighbours(y, z, row, RX, P)
    assert up.tolist() == [-1, 2, -1, -1, 5, -1]
    assert dn.tolist() == [-1, 0, -1, -1, 3, -1]


def nonuniform_rows():
    # rows 10, 11, 12 at x = 100, 101, 104: the middle row sits a quarter of
    # the way from row 10 to row 12
    rx = RX.copy()
    rx[10], rx[11], rx[12] = 100.0, 101.0, 104.0
    return rx


@pytest.mark.parametrize("dy_up,linked", [(1.6, True), (1.9, False)])
def test_chord_weight_on_up_hit(dy_up, linked):
    """The chord from the down hit k to the up hit j is evaluated at x_r, so an
    offset of the up hit moves it by a quarter here: residual (0.25 * dy)^2,
    inside 0.2 cm^2 for 1.6 cm, outside for 1.9 cm."""
    rx = nonuniform_rows()
    hits = [(10, 0.0, 0.0), (11, 0.0, 0.0), (12, dy_up, 0.0)]
    y, z, row, _ = sector(hits, rx)
    up, dn = oracle.neighbours(y, z, row, rx, P)
    assert (up[1] == 2 and dn[1] == 0) == linked
    if not linked:
        assert up[1] == -1 and dn[1] == -1


@pytest.mark.parametrize("dz_dn,linked", [(0.55, True), (0.62, False)])
def test_chord_weight_on_down_hit(dz_dn, linked):
    """A down-hit offset moves the chord at x_r by three quarters."""
    rx = nonuniform_rows()
    hits = [(10, 0.0, dz_dn), (11, 0.0, 0.0), (12, 0.0, 0.0)]
    y, z, row, _ = sector(hits, rx)
    up, dn = oracle.neighbours(y, z, row, rx, P)
    assert (up[1] == 2 and dn[1] == 0) == linked


@pytest.mark.parametrize("off,linked", [(2.95, True), (3.05, False)])
def test_window_around_the_ray_from_the_origin(off, linked):
    """Up and down candidates offset by +off / -off around the ray through the
    middle hit: the chord passes exactly through the hit (score 0), so only the
    window of +-3 cm around the ray prediction y * x_{r+-1} / x_r decides."""
    r = 70
    a = 0.15
    hits = [(r - 1, RX[r - 1] * a - off, 50.0 * RX[r - 1] / RX[r]), (r, RX[r] * a, 50.0),
            (r + 1, RX[r + 1] * a + off, 50.0 * RX[r + 1] / RX[r])]
    y, z, row, _ = sector(hits, RX)
    up, dn = oracle.neighbours(y, z, row, RX, P, "f64")
    assert (up[1] == 2 and dn[1] == 0) == linked


def tie_rows():
    rx = RX.copy()
    rx[29], rx[30], rx[31] = 100.0, 101.0, 102.0  # chord weight exactly 1/2
    return rx


def test_ties_go_to_the_smaller_up_index():
    """Two mirror-image pairs through the hit, both with score exactly 0."""
    rx = tie_rows()
    hits = [(29, 0.25, 0.0), (29, -0.25, 0.0), (30, 0.0, 0.0), (31, -0.25, 0.0), (31, 0.25, 0.0)]
    y, z, row, _ = sector(hits, rx)
    for mode in ("f32", "f64"):
        up, dn = oracle.neighbours(y, z, row, rx, P, mode)
        # (j=3, k=0) and (j=4, k=1) both score 0
        assert up[2] == 3 and dn[2] == 0


def test_ties_in_score_and_up_hit_go_to_the_smaller_down_index():
    rx = tie_rows()
    hits = [(29, -0.25, 0.125), (29, -0.25, -0.125), (30, 0.0, 0.0), (31, 0.25, 0.0)]
    y, z, row, _ = sector(hits, rx)
    for mode in ("f32", "f64"):
        up, dn = oracle.neighbours(y, z, row, rx, P, mode)
        assert up[2] == 3 and dn[2] == 0
    hits = [(29, -0.25, -0.125), (29, -0.25, 0.125), (30, 0.0, 0.0), (31, 0.25, 0.0)]
    y, z, row, _ = sector(hits, rx)
    up, dn = oracle.neighbours(y, z, row, rx, P)
    assert up[2] == 3 and dn[2] == 0


def test_best_pair_wins_over_worse_pair():
    r = 100
    hits = [(r - 1, 10.0 * RX[r - 1] / RX[r], 0.0), (r, 10.0, 0.0), (r + 1, 10.0 * RX[r + 1] / RX[r], 0.0),
            (r + 1, 10.0 * RX[r + 1] / RX[r] + 0.4, 0.0)]
    y, z, row, _ = sector(hits, RX)
    up, dn = oracle.neighbours(y, z, row, RX, P)
    assert up[1] == 2 and dn[1] == 0


def test_unsorted_rows_are_rejected():
    with pytest.raises(ValueError):
        oracle.neighbours(np.zeros(2), np.zeros(2), np.array([3, 2]), RX)
    with pytest.raises(ValueError):
        oracle.neighbours(np.zeros(1), np.zeros(1), np.array([159]), RX)


def test_empty_sector():
    up, dn = oracle.neighbours(np.zeros(0), np.zeros(0), np.zeros(0, np.int32), RX)
    assert len(up) == 0 and len(dn) == 0


def test_noise_free_separated_tracks_link_to_their_own_hits():
    """Straight and curved noise-free tracks far apart: every link joins two
    consecutive hits of the same track."""
    tracks = {"q": [1, -1, 1, -1], "pt": [5.0, 2.0, 1.0, 0.5], "eta": [0.1, 0.3, 0.5, 0.7],
              "phi0": [math.radians(a) for a in (4.0, 8.0, 12.0, 16.0)]}
    b = synth.tracks_workload(tracks, sigma=0.0, noise_frac=0.0)
    s = b.sector(0)
    up, dn = oracle.neighbours(s["y"], s["z"], s["row"], b.row_x, P)
    lab, row = s["label"], s["row"]
    has = (row >= 1) & (row <= 157)
    for i in np.flatnonzero(has):
        j, k = up[i], dn[i]
        same = [h for h in range(len(lab)) if lab[h] == lab[i]]
        rows = set(row[same])
        if row[i] + 1 in rows and row[i] - 1 in rows:
            assert j >= 0 and k >= 0
        if j >= 0:
            assert lab[j] == lab[i] and row[j] == row[i] + 1
            assert lab[k] == lab[i] and row[k] == row[i] - 1
