"""Hand-built sectors through the C ABI, every one compared bit for bit with
the oracle (links, cleaned links, start hits, every tracklet field), each
under launch shapes that put the cases on different search structures.

Cases (Sec. 2 item 1, the neighbour links of the cellular automaton; item 2,
the closest cluster per row; Tab. 1, "very local" seeding):
 - exact chi^2 ties of the neighbour finder, built as mirror images in z
   around a middle hit at z = 0 (the two chords are exact negatives in
   binary32 for any chord weight): ties in chi^2 go to the smaller up index,
   ties in (chi^2, up) to the smaller down index;
 - exact distance ties of the following: a track with z = 0 and tan lambda =
   0 keeps z exactly 0, and two clusters at (y, +d) and (y, -d) in a row are
   then at the same distance: the smaller index is taken (one tie per
   sector: taking either cluster moves z off 0 for the rest of the fit);
 - clusters in rows 0 and 158 (never linked by the neighbour finder) reached
   by the following, outward and inward;
 - candidates exactly at the +-3 cm window edge around the ray prediction,
   and one binary32 step inside and outside it;
 - degenerate grids: all hits of a row on one y, on one z, on one point, one
   hit per row; a lattice of hits on 0.5 cm steps (bin and cell edges on
   hits, many exact ties);
 - a track with an empty row inside its chain, and one with a gap longer
   than the miss limit."""
import math

import numpy as np
import pytest

import oracle
import synth
from _harness import compare_sector, gpu_sector, run_gpu

RX = synth.row_x()
A0 = synth.sector_alpha(0)
F32 = np.float32


class HandBatch:
    """Sectors given as lists of (row, y, z); each sector row-sorted (stable)."""

    def __init__(self, sectors, row_x=RX):
        self.row_x = np.asarray(row_x, np.float32)
        ys, zs, rows, offs, self.order = [], [], [], [0], []
        for hits in sectors:
            order = sorted(range(len(hits)), key=lambda i: (hits[i][0], i))
            rows.append(np.array([hits[i][0] for i in order], np.int32))
            ys.append(np.array([hits[i][1] for i in order], np.float32))
            zs.append(np.array([hits[i][2] for i in order], np.float32))
            offs.append(offs[-1] + len(hits))
            self.order.append(order)
        self.y, self.z, self.row = np.concatenate(ys), np.concatenate(zs), np.concatenate(rows)
        self.hit_offset = np.asarray(offs, np.int64)
        self.n_sectors, self.n_hits = len(sectors), int(offs[-1])

    def sector(self, s):
        a, b = int(self.hit_offset[s]), int(self.hit_offset[s + 1])
        return {"y": self.y[a:b], "z": self.z[a:b], "row": self.row[a:b]}

    def local(self, s, i):
        """Sector-local index of the i-th hit as given."""
        return self.order[s].index(i)


def ties_nf():
    """Rows 59-61: mirrored up/down pairs (tie in chi^2); rows 99-101: one up
    hit on the ray, mirrored down hits (tie in chi^2 and up index)."""
    h = []
    y0 = F32(10.0)
    fu, fd = F32(RX[61]) / F32(RX[60]), F32(RX[59]) / F32(RX[60])
    h += [(60, y0, 0.0),
          (61, y0 * fu + F32(0.1), 0.3), (61, y0 * fu + F32(0.1), -0.3),      # given 1, 2
          (59, y0 * fd - F32(0.1), -0.3), (59, y0 * fd - F32(0.1), 0.3)]      # given 3, 4
    y1 = F32(-7.5)
    fu, fd = F32(RX[101]) / F32(RX[100]), F32(RX[99]) / F32(RX[100])
    h += [(100, y1, 0.0), (101, y1 * fu, 0.0),                                # given 5, 6
          (99, y1 * fd + F32(0.05), 0.4), (99, y1 * fd + F32(0.05), -0.4)]    # given 7, 8
    return h


def track_hits(q, pt, eta, phi0, **kw):
    b = synth.tracks_workload({"q": [q], "pt": [pt], "eta": [eta], "phi0": [phi0]}, sigma=0.0, noise_frac=0.0,
                              **kw)
    s = b.sector(0)
    return [(int(r), float(y), float(z)) for r, y, z in zip(s["row"], s["y"], s["z"])]


def ties_following(r_tie):
    """A z = 0 track over every row with its cluster in row r_tie replaced by
    the mirrored pair (y, +-0.05).  Every other cluster has z = 0, so the
    state's z is exactly 0 until the pair is reached (row 158: outward; row
    0: inward, after the back-transport from row 158; row 120: inside the seed
    chain, where the neighbour finder's tie decides)."""
    h = track_hits(1, 4.0, 0.0, A0 + math.radians(2.0))
    rows = {r: (y, z) for r, y, z in h}
    assert set(rows) == set(range(159)) and all(z == 0.0 for _, z in rows.values())
    out = [(r, y, z) for r, y, z in h if r != r_tie]
    y = rows[r_tie][0]
    return out + [(r_tie, y, 0.05), (r_tie, y, -0.05)]


def window_edges():
    """Candidates at the window edge (binary32 yu + 3, zu - 3), one step
    inside and one outside, each triplet in its own rows."""
    h = []
    r = 10
    for axis in (0, 1):
        for side in (1.0, -1.0):
            for step in (0, 1, -1):
                mid = (F32(12.0), F32(40.0))
                fu = F32(RX[r + 1]) / F32(RX[r])
                fd = F32(RX[r - 1]) / F32(RX[r])
                up = [mid[0] * fu, mid[1] * fu]
                dn = [mid[0] * fd, mid[1] * fd]
                edge = F32(up[axis] + F32(side * 3.0))
                if step:
                    edge = np.nextafter(edge, F32(step * side * np.inf))
                up[axis] = edge
                # the down hit sits inside its window, opposite, so the chord passes near the middle hit
                dn[axis] = F32(dn[axis] - F32(side * 2.9))
                h += [(r, float(mid[0]), float(mid[1])), (r + 1, float(up[0]), float(up[1])),
                      (r - 1, float(dn[0]), float(dn[1]))]
                r += 4
    return h


def degenerate_rows():
    h = []
    for r in range(20, 30):          # one y for the whole row
        h += [(r, 5.0, 30.0 + 0.7 * k) for k in range(12)]
    for r in range(40, 50):          # one z for the whole row
        h += [(r, -8.0 + 0.9 * k, 70.0) for k in range(12)]
    for r in range(60, 70):          # every hit on one point
        h += [(r, 1.25, 12.5)] * 5
    for r in range(80, 90):          # one hit per row, on a ray
        h.append((r, 0.04 * RX[r], 0.5 * RX[r]))
    return h


def lattice(r0=120, n=21, step=0.5):
    """Rows r0-1 .. r0+1 each holding an n x n lattice of 0.5 cm steps."""
    g = [(-5.0 + step * i, 60.0 + step * k) for i in range(n) for k in range(n)]
    return [(r, y, z) for r in (r0 - 1, r0, r0 + 1) for y, z in g]


def gaps():
    """One track with row 70 empty, one with rows 30-35 empty."""
    a = [t for t in track_hits(-1, 1.5, 0.3, A0 - math.radians(3.0)) if t[0] != 70]
    b = [t for t in track_hits(1, 0.8, 0.6, A0 + math.radians(4.0)) if not 30 <= t[0] <= 35]
    return a + b


TIE_ROWS = (158, 0, 120)


def batch():
    return HandBatch([ties_nf(), window_edges(), degenerate_rows(), lattice(), gaps(), []] +
                     [ties_following(r) for r in TIE_ROWS])


TUNINGS = [
    {"bin_hits": 0.5, "nf_rows": 4, "nf_lds_kb": 64, "nf_block": 256},
    {"bin_hits": 64.0, "nf_rows": 1, "nf_lds_kb": 0, "nf_block": 64, "tc_sync": 1},
    {"bin_hits": 0.25, "nf_rows": 32, "nf_lds_kb": 8, "nf_block": 128, "use_graph": 0, "tc_sync": 1},
    {"bin_hits": 0.5, "nf_rows": 3, "nf_lds_kb": 12, "nf_block": 192, "tc_sync": 1},
]


@pytest.mark.gpu
@pytest.mark.parametrize("k", range(len(TUNINGS)))
def test_hand_built_sectors_match_the_oracle(k):
    from paper_1712_09430_amd import catpc as C
    b = batch()
    p = C.catpc_default_params()
    tr, hits, out, st, n = run_gpu(b, p, tuning=TUNINGS[k])
    assert st == C.CATPC_OK, C.catpc_last_error()
    links, trk = out.links_numpy(), out.tracklets_numpy(n)
    bad = []
    for s in range(b.n_sectors):
        bad += compare_sector(b, s, gpu_sector(b, out, links, trk, s), p)
    assert not bad, "\n".join(bad[:20])

    # the tie-breaks themselves, sector 0 (neighbour finder)
    g = gpu_sector(b, out, links, trk, 0)
    L = lambda i: b.local(0, i)
    assert g["nf_up"][L(0)] == L(1) and g["nf_dn"][L(0)] == L(3)
    assert g["nf_up"][L(5)] == L(6) and g["nf_dn"][L(5)] == min(L(7), L(8))
    # following: each mirrored pair gave the smaller index
    for q, r in enumerate(TIE_ROWS):
        s = 6 + q
        g = gpu_sector(b, out, links, trk, s)
        row = b.sector(s)["row"]
        longest = int(np.argmax(g["n_hits"]))
        pair = np.flatnonzero(row == r)
        assert len(pair) == 2 and g["row_hit"][longest][r] == pair.min(), r
        assert g["n_hits"][longest] == 159


def test_window_edge_cases_are_decided_both_ways():
    """The window-edge sector holds accepted and rejected edge candidates
    (so the comparison above tests both outcomes)."""
    b = batch()
    s = b.sector(1)
    up, dn = oracle.neighbours(s["y"], s["z"], s["row"], b.row_x, oracle.Params(), "f32")
    mids = np.flatnonzero(np.isin(s["row"], np.arange(10, 10 + 4 * 12, 4)))
    linked = (up[mids] >= 0).sum()
    assert 0 < linked < len(mids)
