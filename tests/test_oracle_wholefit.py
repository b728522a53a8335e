"""Whole-fit pins of the tracklet filter (Sec. 2 item 2: fit the seed,
follow it row by row, refine with the simplified Kalman filter): noise-free
helices go through the oracle's own neighbour finding, seeding, chord
initialisation and following, and the fitted parameters at x_ref are compared
with the generator's closed-form truth in the first row.  Plus a geometric pin
of the chord initialisation and a check that the refit's sparse F C F^T is
the dense product.

What the decoupled filter (reading: the transverse and longitudinal blocks
are independent) can and cannot recover on exact data:
 - the transverse block (y, sin phi, q/pT) recovers the truth within the
   parameter tolerance (1e-3 cm; 1e-4 relative, floors 1 and 0.1) over the
   whole pT, eta and charge range;
 - the longitudinal block (z, tan lambda) is a linear fit of the z data with
   the path lengths that the transverse state gave at each step.  Early steps
   take them from a state that is still converging (q/pT starts at 0), so z
   carries an error proportional to tan lambda: exactly zero at eta = 0, the
   same Delta z / tan lambda at every eta (up to the binary32 rounding of
   the hit coordinates), within 1e-3 cm and 1e-4 in tan lambda on tracks
   crossing every row; on the shorter low-pT tracks that leave the sector
   before the last row (pT <= 0.35 GeV here) it reaches 1.5e-2 cm * tan lambda
   in z and 2.3e-4 * tan lambda in tan lambda.  That is a named exception with
   its own bound (2e-2 and 5e-4 times tan lambda), not a widened gate: the
   tracks crossing every row are held to the gate."""
import math

import numpy as np
import pytest

import oracle
import synth

P = oracle.Params()
PTS = [float(v) for v in np.exp(np.linspace(math.log(0.2), math.log(10.0), 8))]
ETAS = (0.0, 0.45, 0.85)
A0 = synth.sector_alpha(0)

TOL_Y, TOL_REL = 1e-3, 1e-4
FLOOR = {2: 1.0, 3: 1.0, 4: 0.1}


def _phi_for(q, pt):
    """Launch angle that keeps the helix inside sector 0 for the most rows."""
    best = None
    for d in range(-30, 31, 2):
        phi = A0 + math.radians(d)
        b = synth.tracks_workload({"q": [q], "pt": [pt], "eta": [0.45], "phi0": [phi]}, sigma=0.0,
                                  noise_frac=0.0, truth=True)
        if best is None or b.n_hits > best[0]:
            best = (b.n_hits, phi)
    return best[1]


def _fit(q, pt, eta, phi, **kw):
    b = synth.tracks_workload({"q": [q], "pt": [pt], "eta": [eta], "phi0": [phi]}, sigma=0.0, noise_frac=0.0,
                              truth=True, **kw)
    s = b.sector(0)
    o = oracle.track_sector(s["y"], s["z"], s["row"], b.row_x, P, "f64")
    return b, s, o


def _truth(s, o, t, q, pt, eta):
    h = o["row_hit"][t][o["first_row"][t]]
    return np.array([s["y_true"][h], s["z_true"][h], s["sinphi_true"][h], math.sinh(eta), q / pt])


def _transverse_ok(d, truth):
    assert abs(d[0]) <= TOL_Y, ("y", d[0])
    for k in (2, 4):
        assert abs(d[k]) <= TOL_REL * max(abs(truth[k]), FLOOR[k]), (k, d[k], truth[k])


@pytest.mark.parametrize("q", [1, -1])
@pytest.mark.parametrize("pt", PTS)
def test_noise_free_helices_are_recovered_from_their_own_seed(q, pt):
    phi = _phi_for(q, pt)
    per_eta = {}
    for eta in ETAS:
        b, s, o = _fit(q, pt, eta, phi)
        assert b.n_hits >= 30
        # one seed, one tracklet holding every hit of the track, valid
        assert len(o["start"]) == 1
        assert o["n_hits"][0] == b.n_hits and o["flags"][0] == oracle.VALID
        truth = _truth(s, o, 0, q, pt, eta)
        assert o["x_ref"][0] == float(b.row_x[o["first_row"][0]])
        d = o["param"][0] - truth
        _transverse_ok(d, truth)
        if eta == 0.0:
            assert d[1] == 0.0 and d[3] == 0.0
        elif o["last_row"][0] == len(b.row_x) - 1 and o["first_row"][0] == 0:
            assert abs(d[1]) <= TOL_Y, ("z", d[1])
            assert abs(d[3]) <= TOL_REL * max(abs(truth[3]), 1.0), ("tan lambda", d[3])
        else:
            assert pt <= 0.4, "only low-pT tracks leave the sector early"
            assert abs(d[1]) <= 2e-2 * truth[3], ("z on a short track", d[1])
            assert abs(d[3]) <= 5e-4 * truth[3], ("tan lambda on a short track", d[3])
        per_eta[eta] = (d, truth)
    # the transverse fit does not see z at all: identical at every eta
    for eta in ETAS[1:]:
        assert np.array_equal(per_eta[eta][0][[0, 2, 4]], per_eta[0.0][0][[0, 2, 4]])
    # the longitudinal error is the path-length effect, linear in tan lambda
    r1 = per_eta[0.45][0][1] / per_eta[0.45][1][3]
    r2 = per_eta[0.85][0][1] / per_eta[0.85][1][3]
    assert abs(r1 - r2) <= 2e-2 * max(abs(r1), abs(r2)) + 2e-6, (r1, r2)
    l1 = per_eta[0.45][0][3] / per_eta[0.45][1][3]
    l2 = per_eta[0.85][0][3] / per_eta[0.85][1][3]
    assert abs(l1 - l2) <= 2e-2 * max(abs(l1), abs(l2)) + 2e-8, (l1, l2)


@pytest.mark.parametrize("n_rows", [40, 320])
@pytest.mark.parametrize("q", [1, -1])
def test_noise_free_helices_on_other_row_counts(n_rows, q):
    """The same pin on other pad-row geometries (n_rows planes between the
    same first and last radii: rows four times sparser, or twice as dense):
    a track crossing every row is one valid tracklet holding all its hits,
    its transverse parameters recover the truth within the gate, z and tan
    lambda are exact at eta = 0 and within the gate at eta = 0.45."""
    for pt in (1.0, 3.0, 10.0):
        phi = _phi_for(q, pt)
        for eta in (0.0, 0.45):
            b, s, o = _fit(q, pt, eta, phi, n_rows=n_rows)
            assert len(b.row_x) == n_rows and b.n_hits == n_rows
            assert len(o["start"]) == 1
            assert o["n_hits"][0] == b.n_hits and o["flags"][0] == oracle.VALID
            assert o["first_row"][0] == 0 and o["last_row"][0] == n_rows - 1
            truth = _truth(s, o, 0, q, pt, eta)
            d = o["param"][0] - truth
            _transverse_ok(d, truth)
            if eta == 0.0:
                assert d[1] == 0.0 and d[3] == 0.0
            else:
                assert abs(d[1]) <= TOL_Y, ("z", d[1])
                assert abs(d[3]) <= TOL_REL * max(abs(truth[3]), 1.0), ("tan lambda", d[3])


def test_inward_pass_recovers_the_truth():
    """A dead pad row (19) splits the seeding: the hits next to it get no
    links (the neighbour finder needs both adjacent rows), so one seed starts
    in row 1 and one in row 21.  The upper seed follows inward through the
    gap down to row 0 (21 rows of inward following after the
    back-transport), the lower one outward across it; both hold every hit and
    both recover the truth at row 0."""
    q, pt, eta = -1, 2.5, 0.3
    b, s, o = _fit(q, pt, eta, A0 + math.radians(2.0), dead_rows=(19, 1))
    assert len(o["start"]) == 2
    starts = sorted(o["start_row"].tolist())
    assert starts == [1, 21]
    for t in range(2):
        assert o["n_hits"][t] == b.n_hits and o["first_row"][t] == 0
        truth = _truth(s, o, t, q, pt, eta)
        d = o["param"][t] - truth
        _transverse_ok(d, truth)
        assert abs(d[1]) <= TOL_Y and abs(d[3]) <= TOL_REL * max(abs(truth[3]), 1.0)


@pytest.mark.parametrize("h0,h1", [((100.0, 2.0, 5.0), (101.0, 3.0, 5.5)),
                                   ((120.0, -4.0, -30.0), (121.25, -5.5, -31.2)),
                                   ((90.0, 0.5, 10.0), (91.0, 0.5, 10.4)),
                                   ((200.0, 7.0, 80.0), (201.0, 7.9, 81.3))])
def test_chord_initialisation_is_the_chord_direction(h0, h1):
    """The seed starts at its first hit with the direction of the chord to
    the second: sin phi is the sine of the chord's azimuth in the bending
    plane and tan lambda the tangent of its dip angle over the transverse
    chord length, taken here from the angles themselves (atan2) rather than
    the filter's expressions.  Steps with |dy| comparable to dx separate the
    transverse chord length from dx."""
    st, rc = oracle.init_state(h0, h1, P)
    assert rc == 0
    dx, dy, dz = (h1[0] - h0[0]), (h1[1] - h0[1]), (h1[2] - h0[2])
    azimuth = math.atan2(dy, dx)
    dip = math.atan2(dz, math.hypot(dx, dy))
    assert st[0] == h0[0] and st[1] == h0[1] and st[2] == h0[2]
    assert abs(st[3] - math.sin(azimuth)) < 1e-14
    assert abs(st[4] - math.tan(dip)) < 1e-14
    assert st[5] == 0.0
    # the seed's first hit is already fitted: its variance in y and z is the
    # cluster variance, the angles and the curvature start diffuse and the
    # blocks uncorrelated (prior diag(sigma_y^2, sigma_z^2, 1, 1, 100))
    s2 = float(np.float32(0.1)) ** 2
    assert np.array_equal(st[6:], [s2, 0.0, 1.0, 0.0, 0.0, 100.0, s2, 0.0, 1.0])


def test_chord_initialisation_refuses_a_steep_chord():
    st, rc = oracle.init_state((100.0, 0.0, 0.0), (100.01, 1.0, 0.0), P)
    assert rc == 1


TRI = {(i, j): (i * (i + 1) // 2 + j if i >= j else j * (j + 1) // 2 + i) for i in range(5) for j in range(5)}


@pytest.mark.parametrize("s0,l,q,step", [(0.3, 0.8, 2.0, 1.03), (-0.5, -0.4, -3.0, -12.0), (0.1, 1.2, 0.7, 30.0),
                                         (0.0, 0.0, 0.0, 5.0)])
def test_refit_covariance_transport_is_the_dense_product(s0, l, q, step):
    """C <- F C F^T of the full refit sums only over the structurally nonzero
    entries of F.  The skipped terms are exact zeros added to running sums
    that start at +0, so on finite covariances the result must equal the
    dense product summed in the same index order, bit for bit.  F is read off
    the transport itself: a unit variance on parameter j comes out as
    column j of F (F has a unit diagonal)."""
    x0, x1 = 150.0, 150.0 + step
    p0 = np.array([4.0, 30.0, s0, l, q])
    F = np.zeros((5, 5))
    for j in range(5):
        C = np.zeros(15)
        C[TRI[j, j]] = 1.0
        _, _, C1, rc = oracle.fullfit_transport(x0, p0, C, x1, P)
        assert rc == 0
        for i in range(5):
            F[i, j] = C1[TRI[i, j]]
    assert np.all(np.diag(F) == 1.0)
    rng = np.random.default_rng(int(abs(step) * 100))
    for _ in range(20):
        A = rng.normal(size=(5, 5)) * rng.uniform(0.01, 10, size=5)
        Cd = A @ A.T
        Cp = np.array([Cd[max(TRI_I[k]), min(TRI_I[k])] for k in range(15)])
        _, _, got, rc = oracle.fullfit_transport(x0, p0, Cp, x1, P)
        assert rc == 0
        M = [[0.0] * 5 for _ in range(5)]
        for i in range(5):
            for j in range(5):
                acc = 0.0
                for k in range(5):
                    acc = acc + F[i, k] * Cp[TRI[k, j]]
                M[i][j] = acc
        want = np.zeros(15)
        for i in range(5):
            for j in range(i + 1):
                acc = 0.0
                for k in range(5):
                    acc = acc + M[i][k] * F[j, k]
                want[TRI[i, j]] = acc
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


TRI_I = {v: k for k, v in TRI.items() if k[0] >= k[1]}
