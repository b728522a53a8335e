"""Pins for the oracle's helix transport and simplified Kalman filter
(Sec. 2 item 2): the closed-form helix of the generator, straight lines at
zero field, and exact linear special cases in which the Kalman filter must
equal regularised least squares (a Kalman filter without process noise is
recursive least squares with the prior as a pseudo-measurement)."""
import math

import numpy as np
import pytest

import oracle
import synth

P = oracle.Params()
RX = synth.row_x()
KB = -0.00299792458 * 0.5
S2 = float(np.float32(0.1)) ** 2  # cluster variance as the filter sees it


def state(x, y, z, s, l, q, cy=(1, 0, 1, 0, 0, 1), cz=(1, 0, 1)):
    return np.array([x, y, z, s, l, q, *cy, *cz], np.float64)


def helix_at_x(qpt, tanl, phi0, alpha, x, bz=0.5):
    lo, hi = 0.0, 600.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if synth.helix_point(qpt, tanl, phi0, bz, alpha, mid)[0] < x:
            lo = mid
        else:
            hi = mid
    return synth.helix_point(qpt, tanl, phi0, bz, alpha, 0.5 * (lo + hi))


def test_transport_matches_closed_form_helix():
    """Random helices, steps of 1-40 cm forward and backward; the only
    approximation is the truncated asin(u)/u series (|u| <= 0.15 here), whose
    remainder bounds the z error."""
    rng = np.random.default_rng(11)
    for _ in range(300):
        qpt = rng.choice([-1, 1]) / math.exp(rng.uniform(math.log(0.2), math.log(10)))
        tanl = math.sinh(rng.uniform(-0.9, 0.9))
        alpha = rng.uniform(0, 2 * math.pi)
        phi0 = alpha + rng.uniform(-0.15, 0.15)
        pa = synth.helix_point(qpt, tanl, phi0, 0.5, alpha, rng.uniform(85, 200))
        step = rng.uniform(1, 40) * rng.choice([-1, 1])
        # exact position at x = pa.x + step
        lo, hi = 0.0, 600.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if synth.helix_point(qpt, tanl, phi0, 0.5, alpha, mid)[0] < pa[0] + step:
                lo = mid
            else:
                hi = mid
        pb = synth.helix_point(qpt, tanl, phi0, 0.5, alpha, 0.5 * (lo + hi))
        st, rc = oracle.propagate(state(pa[0], pa[1], pa[2], pa[3], tanl, qpt), pb[0], P)
        k = KB * qpt
        ch = math.hypot(pb[0] - pa[0], pb[1] - pa[1])
        u = abs(k * ch / 2)
        if abs(u - 0.2) < 1e-6:
            continue
        assert rc == (2 if u > 0.2 else 0)
        if rc:
            continue
        bound = ch * (63 / 2816) * u ** 10 / (1 - u * u) * abs(tanl) + 1e-9
        assert abs(st[1] - pb[1]) < 1e-9
        assert abs(st[3] - pb[3]) < 1e-12
        assert abs(st[2] - pb[2]) < bound


def test_every_series_term_matters():
    """A 40 cm step at pT = 0.2 GeV (u ~ 0.16): the last kept series term
    (35/1152 u^8) moves z by far more than the truncation remainder, and the
    result stays within that remainder, so a wrong or missing coefficient
    would show."""
    qpt, tanl, alpha = 5.0, 1.0, 0.0
    pa = synth.helix_point(qpt, tanl, 0.0, 0.5, alpha, 20.0)
    pb = helix_at_x(qpt, tanl, 0.0, alpha, pa[0] + 40.0)
    st, rc = oracle.propagate(state(pa[0], pa[1], pa[2], pa[3], tanl, qpt), pb[0], P)
    assert rc == 0
    ch = math.hypot(pb[0] - pa[0], pb[1] - pa[1])
    u = abs(KB * qpt * ch / 2)
    bound = ch * (63 / 2816) * u ** 10 / (1 - u * u) * tanl + 1e-10
    assert (35 / 1152) * u ** 8 * ch * tanl > 30 * bound
    assert abs(st[2] - pb[2]) < bound


def test_zero_field_is_a_straight_line():
    p0 = oracle.Params(bz=0.0)
    st0 = state(100.0, 3.0, 20.0, 0.3, 0.7, 2.0)
    st, rc = oracle.propagate(st0, 117.0, p0)
    assert rc == 0
    c = math.sqrt(1 - 0.09)
    assert st[3] == 0.3 and st[5] == 2.0
    assert abs(st[1] - (3.0 + 17.0 * 0.3 / c)) < 1e-12
    assert abs(st[2] - (20.0 + 0.7 * 17.0 / c)) < 1e-12


def test_transport_limits():
    # |sin phi| would reach 0.999: refused, state untouched
    st0 = state(100.0, 0.0, 0.0, 0.99, 0.0, 5.0)
    st, rc = oracle.propagate(st0, 100.0 + (0.999 - 0.99) / (-KB * 5.0) * -1.0 + 5.0, P)
    assert rc in (0, 1)
    st, rc = oracle.propagate(state(100.0, 0.0, 0.0, -0.99, 0.0, 5.0), 105.0, P)
    assert rc == 1 and np.array_equal(st, state(100.0, 0.0, 0.0, -0.99, 0.0, 5.0))
    # arc-series range: |k * chord / 2| > 0.2
    st, rc = oracle.propagate(state(0.0, 0.0, 0.0, 0.0, 0.0, 5.0), 60.0, P)
    assert rc == 2


def make_sector(rows, ys, zs):
    """One hit per listed row; returns arrays plus the hit-per-row list."""
    order = np.argsort(rows, kind="stable")
    rows, ys, zs = np.asarray(rows)[order], np.asarray(ys)[order], np.asarray(zs)[order]
    rh = np.full(159, -1, np.int32)
    rh[rows] = np.arange(len(rows))
    return ys.astype(np.float32), zs.astype(np.float32), rows.astype(np.int32), rh


def lsq(H, m, prior_mean, prior_var, var):
    A = np.diag(1.0 / np.asarray(prior_var)) + H.T @ H / var
    b = np.asarray(prior_mean) / np.asarray(prior_var) + H.T @ m / var
    C = np.linalg.inv(A)
    return C @ b, C


def gapped_rows(rng, r0):
    up = [r for r in range(r0 + 2, 159) if rng.random() > 0.2]
    dn = [r for r in range(0, r0) if rng.random() > 0.3]
    return [r0, r0 + 1] + up, dn


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_longitudinal_block_is_least_squares(seed):
    """y == 0 keeps sin phi and q/pT at exactly 0, so z is exactly linear in
    (z, tan lambda) with arc = dx: the filter (outward, back, inward) must equal
    the regularised straight-line least-squares fit."""
    rng = np.random.default_rng(seed)
    r0 = 50
    above, below = gapped_rows(rng, r0)
    rows = above + below
    x = RX[rows].astype(np.float64)
    zt = 10.0 + 0.6 * (x - x[0])
    zm = (zt + rng.normal(0, 0.1, len(x))).astype(np.float32)
    y, z, row, rh = make_sector(rows, np.zeros(len(rows)), zm)
    o = oracle.refit(y, z, RX, rh[None, :], np.array([r0]), P, "f64")
    assert o["flags"][0] & 1
    x0 = float(RX[r0])
    z0, z1 = float(zm[0]), float(zm[1])
    lam0 = (z1 - z0) / (float(RX[r0 + 1]) - x0)
    meas = list(range(1, len(rows)))
    H = np.stack([np.ones(len(meas)), x[meas] - x0], 1)
    th, C = lsq(H, zm[meas].astype(np.float64), [z0, lam0], [S2, 1.0], S2)
    xf = float(RX[min(rows)])
    F = np.array([[1.0, xf - x0], [0.0, 1.0]])
    thf, Cf = F @ th, F @ C @ F.T
    assert o["x_ref"][0] == xf
    assert abs(o["param"][0, 1] - thf[0]) < 1e-10 and abs(o["param"][0, 3] - thf[1]) < 1e-12
    np.testing.assert_allclose(o["cov"][0, [2, 7, 9]], [Cf[0, 0], Cf[1, 0], Cf[1, 1]], rtol=1e-9)
    assert o["param"][0, 0] == 0 and o["param"][0, 2] == 0 and o["param"][0, 4] == 0


@pytest.mark.parametrize("seed", [4, 5])
def test_transverse_covariance_is_least_squares(seed):
    """Same configuration: the transverse block is the linear model
    y = y0 + s dx + q kb dx^2 / 2, so its covariance must equal the
    least-squares covariance of a parabola with the diffuse prior."""
    rng = np.random.default_rng(seed)
    r0 = 30
    above, below = gapped_rows(rng, r0)
    rows = above + below
    x = RX[rows].astype(np.float64)
    y, z, row, rh = make_sector(rows, np.zeros(len(rows)), 5.0 + 0.2 * (x - x[0]))
    o = oracle.refit(y, z, RX, rh[None, :], np.array([r0]), P, "f64")
    x0 = float(RX[r0])
    meas = list(range(1, len(rows)))
    d = x[meas] - x0
    H = np.stack([np.ones(len(d)), d, KB * d * d / 2], 1)
    _, C = lsq(H, np.zeros(len(d)), [0, 0, 0], [S2, 1.0, 100.0], S2)
    df = float(RX[min(rows)]) - x0
    F = np.array([[1, df, KB * df * df / 2], [0, 1, KB * df], [0, 0, 1]])
    Cf = F @ C @ F.T
    got = o["cov"][0]
    want = {0: Cf[0, 0], 3: Cf[1, 0], 5: Cf[1, 1], 10: Cf[2, 0], 12: Cf[2, 1], 14: Cf[2, 2]}
    for k, v in want.items():
        assert abs(got[k] - v) <= 1e-9 * math.sqrt(abs(Cf[[0, 1, 2][{0: 0, 3: 1, 5: 1, 10: 2, 12: 2, 14: 2}[k]],
                                                         [0, 1, 2][{0: 0, 3: 1, 5: 1, 10: 2, 12: 2, 14: 2}[k]]]
                                                      * Cf[[0, 0, 1, 0, 1, 2][[0, 3, 5, 10, 12, 14].index(k)],
                                                           [0, 0, 1, 0, 1, 2][[0, 3, 5, 10, 12, 14].index(k)]])) + 1e-18
    for k in (1, 4, 6, 8, 11, 13):  # cross-block terms stay zero
        assert got[k] == 0


def test_transverse_state_is_least_squares_in_the_linear_regime():
    """Nearly straight, nearly radial track with tiny measurement scatter: the
    transverse model is linear up to O(sin^3 phi) terms, so the filtered
    (y, sin phi, q/pT) must agree with the least-squares parabola."""
    rng = np.random.default_rng(9)
    r0 = 40
    above, below = gapped_rows(rng, r0)
    rows = above + below
    x = RX[rows].astype(np.float64)
    x0 = float(RX[r0])
    d = x - x0
    qt = 0.02
    yt = 0.3 + 1e-3 * d + KB * qt * d * d / 2
    ym = (yt + rng.normal(0, 1e-3, len(x))).astype(np.float32)
    y, z, row, rh = make_sector(rows, ym, np.zeros(len(rows)))
    o = oracle.refit(y, z, RX, rh[None, :], np.array([r0]), P, "f64")
    yv = ym.astype(np.float64)
    s_init = (yv[1] - yv[0]) / math.hypot(float(RX[r0 + 1]) - x0, yv[1] - yv[0])
    meas = list(range(1, len(rows)))
    dm = d[meas]
    H = np.stack([np.ones(len(dm)), dm, KB * dm * dm / 2], 1)
    th, _ = lsq(H, yv[meas], [yv[0], s_init, 0.0], [S2, 1.0, 100.0], S2)
    df = float(RX[min(rows)]) - x0
    F = np.array([[1, df, KB * df * df / 2], [0, 1, KB * df], [0, 0, 1]])
    thf = F @ th
    got = o["param"][0]
    assert abs(got[0] - thf[0]) < 2e-6
    assert abs(got[2] - thf[1]) < 2e-8
    assert abs(got[4] - thf[2]) < 2e-5
    # and the estimate is close to the truth (noise 1e-3 cm)
    assert abs(got[4] - qt) < 5e-3


def test_truth_is_a_fixed_point():
    """Starting exactly on a helix, transporting row by row and updating with
    noise-free clusters leaves the state on the helix."""
    qpt, tanl, phi0, alpha = -2.5, 0.5, 0.05, 0.0
    pts = [helix_at_x(qpt, tanl, phi0, alpha, float(x)) for x in RX[:120]]
    st = state(pts[0][0], pts[0][1], pts[0][2], pts[0][3], tanl, qpt, cy=(S2, 0, 0.01, 0, 0, 1), cz=(S2, 0, 0.01))
    for p in pts[1:]:
        st, rc = oracle.propagate(st, p[0], P)
        assert rc == 0
        st, rc = oracle.update(st, p[1], p[2], P)
        assert rc == 0
        assert abs(st[1] - p[1]) < 1e-9 and abs(st[2] - p[2]) < 1e-9 and abs(st[3] - p[3]) < 1e-11
    assert abs(st[5] - qpt) < 1e-9 and abs(st[4] - tanl) < 1e-11


def test_update_matches_scalar_kalman_gain():
    """One update against the textbook gain K = C H^T / (H C H^T + R) on a
    random positive-definite transverse block."""
    rng = np.random.default_rng(3)
    A = rng.normal(size=(3, 3))
    Cy = A @ A.T + 0.1 * np.eye(3)
    B = rng.normal(size=(2, 2))
    Cz = B @ B.T + 0.1 * np.eye(2)
    st0 = state(100, 1.0, 2.0, 0.1, 0.2, 0.3, cy=(Cy[0, 0], Cy[1, 0], Cy[1, 1], Cy[2, 0], Cy[2, 1], Cy[2, 2]),
                cz=(Cz[0, 0], Cz[1, 0], Cz[1, 1]))
    st, rc = oracle.update(st0, 1.5, 1.7, P)
    assert rc == 0
    Ky = Cy[:, 0] / (Cy[0, 0] + S2)
    Kz = Cz[:, 0] / (Cz[0, 0] + S2)
    np.testing.assert_allclose(st[[1, 3, 5]], np.array([1.0, 0.1, 0.3]) + Ky * 0.5, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(st[[2, 4]], np.array([2.0, 0.2]) - Kz * 0.3, rtol=1e-14, atol=1e-14)
    Cy1 = Cy - np.outer(Ky, Cy[0, :])
    Cz1 = Cz - np.outer(Kz, Cz[0, :])
    np.testing.assert_allclose(st[[6, 7, 8, 9, 10, 11]], [Cy1[0, 0], Cy1[1, 0], Cy1[1, 1], Cy1[2, 0], Cy1[2, 1],
                                                         Cy1[2, 2]], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(st[[12, 13, 14]], [Cz1[0, 0], Cz1[1, 0], Cz1[1, 1]], rtol=1e-12, atol=1e-14)


def test_spd_check():
    good = state(100, 0, 0, 0, 0, 0, cy=(1.0, 0.5, 1.0, 0.2, 0.1, 1.0), cz=(1.0, 0.3, 1.0))
    assert oracle.spd(good) and oracle.spd(good, "f32")
    bad = good.copy()
    bad[7] = 1.5  # |c_sy| > sqrt(c_yy c_ss)
    assert not oracle.spd(bad) and not oracle.spd(bad, "f32")
    bad = good.copy()
    bad[14] = -0.1
    assert not oracle.spd(bad)
    bad = good.copy()
    bad[11] = float("nan")
    assert not oracle.spd(bad)


def test_covariance_stays_positive_definite_along_real_fits():
    b = synth.sector_workload(seed=4)
    s = b.sector(0)
    o = oracle.track_sector(s["y"], s["z"], s["row"], b.row_x, P, "f64")
    assert not np.any(o["flags"] & oracle.SPD_FAIL)
    for c in o["cov"]:
        Cy = np.array([[c[0], c[3], c[10]], [c[3], c[5], c[12]], [c[10], c[12], c[14]]])
        Cz = np.array([[c[2], c[7]], [c[7], c[9]]])
        assert np.all(np.linalg.eigvalsh(Cy) > 0) and np.all(np.linalg.eigvalsh(Cz) > 0)
