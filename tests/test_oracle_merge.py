"""Pins for the oracle's merging of track segments inside a sector (Sec. 2
item 3: segments of one track that the following split at a gap are merged
before the sector-border merging).  Exact helix states (closed form of a
helix in a constant field, written here independently of the filter's
transport) make the transported difference vanish, so the 5-parameter chi^2
reduces to closed forms: with no covariance on the outer segment's side it is
sum(d_i^2 / sigma_i^2); with covariance it is d^T (J C J^T + C_B)^-1 d with
the Jacobian J of the exact helix map taken by finite differences.  The
mutual-best rule, its tie break, the gap, window and chi^2 cuts and the
degenerate cases are checked on hand-built segments; on generated events
with a dead band of pad rows the links found agree with the generator's
track labels."""
import math

import numpy as np
import pytest

import oracle
import synth
from _harness import chains, oracle_merge_sector

P = oracle.Params()
RX = synth.row_x()
KB = -0.00299792458 * P.bz
TRI = [(i, j) for i in range(5) for j in range(i + 1)]


def helix(x, q, s0=None, tanl=0.4):
    """State (y, z, sin phi, tan lambda, q/pT) at x of the helix through the
    origin with sin phi = s0 there (closed form); by default s0 puts
    sin phi = 0 at x = 166 cm, the middle of the pad rows."""
    k = KB * q
    s0 = -k * 166.0 if s0 is None else s0
    s = s0 + k * x
    y = (math.sqrt(1 - s0 * s0) - math.sqrt(1 - s * s)) / k
    z = tanl * (math.asin(s) - math.asin(s0)) / k
    return np.array([y, z, s, tanl, q])


def helix_map(x0, st, x1):
    """The exact helix map of a state from x0 to x1."""
    y, z, s, l, q = st
    k = KB * q
    s1 = s + k * (x1 - x0)
    return np.array([y + (math.sqrt(1 - s * s) - math.sqrt(1 - s1 * s1)) / k,
                     z + l * (math.asin(s1) - math.asin(s)) / k, s1, l, q])


def packed(M):
    return np.array([M[i, j] for i, j in TRI], np.float32)


def segments(specs):
    """specs: list of (ok, a_last, end state, end cov, b_first, start state, start cov)."""
    cols = list(zip(*specs))
    ok = np.array(cols[0], np.int32)
    a_last, b_first = np.array(cols[1], np.int32), np.array(cols[4], np.int32)
    e_x = np.array([RX[r] for r in a_last], np.float32)
    s_x = np.array([RX[r] for r in b_first], np.float32)
    e_p = np.array(cols[2], np.float32)
    s_p = np.array(cols[5], np.float32)
    e_C = np.array([packed(c) for c in cols[3]])
    s_C = np.array([packed(c) for c in cols[6]])
    return ok, a_last, e_x, e_p, e_C, b_first, s_x, s_p, s_C


SIG = np.array([0.1, 0.1, 0.01, 0.01, 0.05])
CB = np.diag(SIG ** 2)
ZERO = np.zeros((5, 5))


def seg(q, a_last, b_first, d_end=(0, 0, 0, 0, 0), d_start=(0, 0, 0, 0, 0), CA=ZERO, CBm=CB, ok=1, s0=None):
    """One segment ending at row a_last (state: exact + d_end) whose tracklet
    starts at row b_first (state: exact + d_start)."""
    return (ok, a_last, helix(float(RX[a_last]), q, s0) + np.array(d_end), CA, b_first,
            helix(float(RX[b_first]), q, s0) + np.array(d_start), CBm)


def run(specs, mp=None):
    return oracle.merge(RX, *segments(specs), P, mp)


@pytest.mark.parametrize("q", [0.2, 1.0, -3.0])
@pytest.mark.parametrize("comp", range(5))
def test_chi2_closed_form_without_inner_covariance(q, comp):
    """C_A = 0: chi^2 = d^2 / sigma^2 for an offset d of one start parameter."""
    d = np.zeros(5)
    d[comp] = 3.0 * SIG[comp]
    # segment 0 ends at row 40; segment 1 (same helix) starts at row 49
    specs = [seg(q, 40, 10), seg(q, 120, 49, d_start=d)]
    nxt, chi2 = run(specs)
    assert nxt[0] == 1 and nxt[1] == -1
    assert chi2[0] == pytest.approx(9.0, rel=2e-3)


@pytest.mark.parametrize("q,s0", [(0.5, 0.1), (-2.0, -0.2), (4.0, None)])
def test_chi2_with_inner_covariance_uses_the_helix_jacobian(q, s0):
    rng = np.random.default_rng(int(abs(q) * 10))
    G = rng.normal(size=(5, 5)) * np.array([0.05, 0.05, 0.004, 0.004, 0.02])
    CA = G @ G.T + np.diag([1e-3, 1e-3, 1e-6, 1e-6, 1e-4])
    a_last, b_first = 30, 52
    d = np.array([0.05, -0.04, 0.003, -0.002, 0.01])
    specs = [seg(q, a_last, 5, CA=CA, s0=s0), seg(q, 150, b_first, d_start=d, s0=s0)]
    nxt, chi2 = run(specs)
    # the exact helix map's Jacobian by central differences
    x0, x1 = float(np.float32(RX[a_last])), float(np.float32(RX[b_first]))
    st = np.array(specs[0][2], np.float32).astype(np.float64)
    J = np.zeros((5, 5))
    for j in range(5):
        h = 1e-6 * max(1.0, abs(st[j]))
        e = np.zeros(5)
        e[j] = h
        J[:, j] = (helix_map(x0, st + e, x1) - helix_map(x0, st - e, x1)) / (2 * h)
    CAf = np.zeros((5, 5))
    for (i, j), v in zip(TRI, packed(CA)):
        CAf[i, j] = CAf[j, i] = v
    CBf = np.zeros((5, 5))
    for (i, j), v in zip(TRI, packed(CB)):
        CBf[i, j] = CBf[j, i] = v
    diff = np.array(specs[1][5], np.float32).astype(np.float64) - helix_map(x0, st, x1)
    want = diff @ np.linalg.solve(J @ CAf @ J.T + CBf, diff)
    assert nxt[0] == 1
    assert chi2[0] == pytest.approx(want, rel=2e-3)
    # a dropped covariance term would move chi^2 well beyond that
    assert not (diff @ np.linalg.solve(CBf, diff) == pytest.approx(want, rel=0.05))


def test_mutual_best_and_tie_break():
    dy = np.array([0.2, 0, 0, 0, 0])
    # two inner segments, one continuation: the continuation keeps the closer one
    nxt, chi2 = run([seg(1.0, 40, 5, d_end=dy), seg(1.0, 40, 6, d_end=dy / 2), seg(1.0, 140, 49)])
    assert list(nxt) == [-1, 2, -1]
    assert chi2[1] == pytest.approx(1.0, rel=2e-3) and chi2[0] == -1
    # one inner segment, two continuations: the closer one
    nxt, _ = run([seg(1.0, 40, 5), seg(1.0, 140, 49, d_start=dy), seg(1.0, 140, 50, d_start=dy / 2)])
    assert list(nxt) == [2, -1, -1]
    # identical inner segments: the smaller index
    s = seg(1.0, 40, 5, d_end=dy)
    nxt, _ = run([seg(1.0, 140, 49), s, s])
    assert list(nxt) == [-1, 0, -1]
    # identical continuations: the smaller index
    t = seg(1.0, 140, 49, d_start=dy)
    nxt, _ = run([seg(1.0, 40, 5), t, t])
    assert list(nxt) == [1, -1, -1]
    # a chain of three segments across two gaps
    nxt, _ = run([seg(1.0, 40, 5), seg(1.0, 90, 49), seg(1.0, 150, 99)])
    assert list(nxt) == [1, 2, -1]
    prev, head = chains(nxt)
    assert list(prev) == [-1, 0, 1] and list(head) == [0, 0, 0]


@pytest.mark.parametrize("gap,linked", [(0, False), (1, True), (30, True), (31, False), (-5, False)])
def test_gap_rule(gap, linked):
    nxt, _ = run([seg(1.0, 60, 5), seg(1.0, 150, 60 + gap)])
    assert (nxt[0] == 1) == linked
    mp = oracle.MergeParams(max_gap=max(gap - 1, 0))
    assert run([seg(1.0, 60, 5), seg(1.0, 150, 60 + gap)], mp)[0][0] == -1


@pytest.mark.parametrize("off,linked", [(9.0, True), (11.0, False), (-9.0, True), (-11.0, False)])
@pytest.mark.parametrize("comp", [0, 1])
def test_straight_line_window(off, linked, comp):
    """sin phi = 0.5 at the end of the inner segment and a 25-row gap: the
    straight line moves 14 cm in y and 11.5 cm in z (about 0.15 cm of
    sagitta at 5 GeV), so the window is tested along the track's direction."""
    d = np.zeros(5)
    d[comp] = off
    wide = np.diag([1e4, 1e4, 1e-4, 1e-4, 1e-2])
    q = 0.2
    s0 = 0.5 - KB * q * float(RX[60])
    nxt, _ = run([seg(q, 60, 5, s0=s0), seg(q, 150, 85, d_start=d, CBm=wide, s0=s0)])
    assert (nxt[0] == 1) == linked


@pytest.mark.parametrize("c2,linked", [(24.0, True), (26.0, False)])
def test_chi2_cut(c2, linked):
    d = np.array([math.sqrt(c2) * SIG[0], 0, 0, 0, 0])
    nxt, chi2 = run([seg(1.0, 60, 5), seg(1.0, 150, 70, d_start=d)])
    assert (nxt[0] == 1) == linked
    mp = oracle.MergeParams(chi2_max=c2 - 1.0 if linked else c2 + 1.0)
    assert (run([seg(1.0, 60, 5), seg(1.0, 150, 70, d_start=d)], mp)[0][0] == 1) != linked


def test_degenerate_cases():
    # a segment whose refit did not finish takes part in nothing
    assert list(run([seg(1.0, 60, 5, ok=0), seg(1.0, 150, 70)])[0]) == [-1, -1]
    assert list(run([seg(1.0, 60, 5), seg(1.0, 150, 70, ok=0)])[0]) == [-1, -1]
    # V not positive definite
    bad = np.diag([0.01, -0.01, 1e-4, 1e-4, 1e-2])
    assert list(run([seg(1.0, 60, 5), seg(1.0, 150, 70, CBm=bad)])[0]) == [-1, -1]
    # a transport that turns the track past |sin phi| = 0.999 breaks the link
    # (sin phi grows by about 0.0015 per row for q/pT = -1)
    turning = (1, 60, np.array([0.0, 0.0, 0.995, 0.4, -1.0]), ZERO, 5, helix(float(RX[5]), -1.0), CB)
    beyond = (1, 150, np.array([0.0, 0.0, 0.995, 0.4, -1.0]), ZERO, 70, np.array([0.0, 0.0, 0.99, 0.4, -1.0]),
              np.diag([1e8, 1e8, 1.0, 1.0, 1.0]))
    assert list(run([turning, beyond], oracle.MergeParams(window=1e6, chi2_max=1e30))[0]) == [-1, -1]
    near = (1, 150, np.array([0.0, 0.0, 0.995, 0.4, -1.0]), ZERO, 62, np.array([0.0, 0.0, 0.99, 0.4, -1.0]),
            np.diag([1e8, 1e8, 1.0, 1.0, 1.0]))
    assert list(run([turning, near], oracle.MergeParams(window=1e6, chi2_max=1e30))[0]) == [1, -1]
    # empty input
    nxt, chi2 = oracle.merge(RX, *[np.zeros((0,) + sh, dt) for sh, dt in
                                   [((), np.int32), ((), np.int32), ((), np.float32), ((5,), np.float32),
                                    ((15,), np.float32), ((), np.int32), ((), np.float32), ((5,), np.float32),
                                    ((15,), np.float32)]], P)
    assert len(nxt) == 0 and len(chi2) == 0


def test_dead_band_splits_are_merged_by_label():
    """Generated events with 8 dead pad rows: the tracklet following loses
    the track across the band (more than 4 missed rows) and the merge joins
    the two segments.  Against the generator's labels: at least 95 % of the
    labels found as two segments are linked, and links between different
    labels stay below 1 %."""
    b = synth.event_workload(seed=4, n_tracks=4000, dead_rows=(70, 8))
    split = linked = fake = links = 0
    for s in (0, 7, 20, 33):
        nxt, chi2, lab = oracle_merge_sector(b, s, P)
        labs, cnt = np.unique(lab[lab >= 0], return_counts=True)
        split += int(np.sum(cnt == 2))
        for a in np.flatnonzero(nxt >= 0):
            links += 1
            if lab[a] == lab[nxt[a]]:
                linked += 1
            else:
                fake += 1
        assert np.all((chi2 >= 0) == (nxt >= 0)) and np.all(chi2[nxt >= 0] <= 25.0)
    assert split > 200
    assert linked >= 0.95 * split
    assert fake <= 0.01 * links


def test_no_links_without_gaps():
    b = synth.sector_workload(seed=2, n_tracks=300)
    nxt, _, lab = oracle_merge_sector(b, 0, P)
    for a in np.flatnonzero(nxt >= 0):
        assert lab[a] == lab[nxt[a]]
    assert np.sum(nxt >= 0) <= 3
