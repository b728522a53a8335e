"""Pins for the oracle's full Kalman refit (Sec. 2 item 4: the final fit
with the full Kalman filter): noise-free helices are reproduced exactly; at
zero field a straight track's full covariance equals the least-squares
covariance of the linear model with the prior (a Kalman filter without
process noise is recursive least squares); with tan(lambda) = 0 the coupling
terms vanish and the fit equals the decoupled filter of the tracklet
construction; on smeared tracks all five pulls and chi^2/ndf are standard."""
import math

import numpy as np
import pytest

import oracle
import synth

P = oracle.Params()
RX = synth.row_x()
S2 = float(np.float32(0.1)) ** 2  # cluster variance as the filter sees it
TRI = {(i, j): (i * (i + 1) // 2 + j if i >= j else j * (j + 1) // 2 + i) for i in range(5) for j in range(5)}


def unpack(c):
    return np.array([[c[TRI[i, j]] for j in range(5)] for i in range(5)])


def track_hits(b, label=None):
    s = b.sector(0)
    rows = s["row"]
    sel = np.ones(len(rows), bool) if label is None else s["label"] == label
    idx = np.flatnonzero(sel)
    return rows[idx], s["y"][idx], s["z"][idx], s, idx


@pytest.mark.parametrize("q,pt,eta,phi", [(1, 8.0, 0.1, 3.0), (-1, 1.0, 0.5, 9.0), (1, 0.35, 0.8, 14.0),
                                          (-1, 0.5, 0.65, 6.0)])
def test_noise_free_helices_are_reproduced(q, pt, eta, phi):
    b = synth.tracks_workload({"q": [q], "pt": [pt], "eta": [eta], "phi0": [math.radians(phi)]}, sigma=0.0,
                              noise_frac=0.0, truth=True)
    rows, hy, hz, s, idx = track_hits(b)
    i0 = idx[0]
    start = [s["y_true"][i0], s["z_true"][i0], s["sinphi_true"][i0], math.sinh(eta), q / pt]
    r = oracle.fullfit(RX, rows, hy, hz, RX[rows[0]], start, rows[0], P, "f64")
    assert r["flags"] == 1 and r["ndf"] == 2 * len(rows) - 5
    assert r["chi2"] < 1e-4
    last = idx[-1]
    assert abs(r["param"][0] - s["y_true"][last]) < 2e-4
    assert abs(r["param"][1] - s["z_true"][last]) < 2e-4
    assert abs(r["param"][2] - s["sinphi_true"][last]) < 1e-5
    assert abs(r["param"][3] - math.sinh(eta)) < 1e-5
    assert abs(r["param"][4] - q / pt) < 1e-4 * max(1.0, abs(q / pt))


def test_zero_field_covariance_is_least_squares():
    p0 = oracle.Params(bz=0.0)
    rng = np.random.default_rng(3)
    rows = np.sort(rng.choice(np.arange(10, 150), 40, replace=False)).astype(np.int32)
    zeros = np.zeros(len(rows))
    r = oracle.fullfit(RX, rows, zeros, zeros, RX[rows[0]], [0, 0, 0, 0, 0.7], rows[0], p0, "f64")
    assert r["flags"] == 1
    x = RX[rows].astype(np.float64)
    d0 = x[0] - x[-1]
    # information of the parameters at the last hit: prior at the first hit plus every hit
    J = np.eye(5)
    J[0, 2] = d0
    J[1, 3] = d0
    info = J.T @ np.diag(1.0 / np.array([S2, S2, 1.0, 1.0, 100.0])) @ J
    for xi in x:
        hy = np.array([1.0, 0, xi - x[-1], 0, 0])
        hz = np.array([0, 1.0, 0, xi - x[-1], 0])
        info += np.outer(hy, hy) / S2 + np.outer(hz, hz) / S2
    want = np.linalg.inv(info)
    got = unpack(r["cov"])
    scale = np.sqrt(np.outer(np.diag(want), np.diag(want)))
    assert np.all(np.abs(got - want) <= 1e-9 * scale)


def test_zero_field_state_is_least_squares_in_the_linear_regime():
    p0 = oracle.Params(bz=0.0)
    rng = np.random.default_rng(4)
    rows = np.arange(20, 120, 2).astype(np.int32)
    x = RX[rows].astype(np.float64)
    hy = (1e-4 * rng.standard_normal(len(rows))).astype(np.float32)
    hz = (2.0 + 0.001 * (x - x[0]) + 1e-4 * rng.standard_normal(len(rows))).astype(np.float32)
    r = oracle.fullfit(RX, rows, hy, hz, RX[rows[0]], [0, 2.0, 0, 0, 0], rows[0], p0, "f64")
    d = x - x[-1]
    # least squares of y = y_N + d s and z = z_N + d l with the prior at the first hit
    A = np.zeros((2 * len(rows) + 5, 5))
    bvec = np.zeros(2 * len(rows) + 5)
    w = np.zeros(len(bvec))
    A[:len(rows), 0], A[:len(rows), 2] = 1, d
    A[len(rows):2 * len(rows), 1], A[len(rows):2 * len(rows), 3] = 1, d
    bvec[:len(rows)], bvec[len(rows):2 * len(rows)] = hy, hz
    w[:2 * len(rows)] = 1 / S2
    pr = 2 * len(rows)
    A[pr, [0, 2]] = 1, d[0]
    A[pr + 1, [1, 3]] = 1, d[0]
    A[pr + 2, 2] = A[pr + 3, 3] = A[pr + 4, 4] = 1
    bvec[pr + 1] = 2.0
    w[pr:] = 1 / np.array([S2, S2, 1.0, 1.0, 100.0])
    theta = np.linalg.solve(A.T @ (w[:, None] * A), A.T @ (w * bvec))
    assert np.allclose(r["param"][:4], theta[:4], rtol=0, atol=1e-7)


def test_tan_lambda_zero_reduces_to_the_decoupled_filter():
    b = synth.tracks_workload({"q": [1], "pt": [0.8], "eta": [0.0], "phi0": [math.radians(8.0)]}, sigma=0.0,
                              noise_frac=0.0, truth=True)
    rows, hy, hz, s, idx = track_hits(b)
    assert np.all(hz == 0)
    i0 = idx[0]
    start = [s["y_true"][i0] + 0.05, 0.0, s["sinphi_true"][i0] + 0.01, 0.0, 1.0]
    full = oracle.fullfit(RX, rows, hy, hz, RX[rows[0]], start, rows[0], P, "f64")
    # the decoupled filter of the tracklet construction, stepped along the same rows
    st = np.array([RX[rows[0]], start[0], 0.0, start[2], 0.0, start[4], S2, 0, 1, 0, 0, 100, S2, 0, 1],
                  np.float64)
    k = 0
    for r in range(rows[0], rows[-1] + 1):
        if r > rows[0]:
            st, rc = oracle.propagate(st, RX[r], P)
            assert rc == 0
        if k < len(rows) and rows[k] == r:
            st, rc = oracle.update(st, hy[k], hz[k], P)
            assert rc == 0
            k += 1
    C = unpack(full["cov"])
    pairs = {6: (0, 0), 7: (2, 0), 8: (2, 2), 9: (4, 0), 10: (4, 2), 11: (4, 4), 12: (1, 1), 13: (3, 1), 14: (3, 3)}
    for slot, (i, j) in pairs.items():
        assert abs(C[i, j] - st[slot]) <= 1e-10 * math.sqrt(C[i, i] * C[j, j])
    assert np.allclose(full["param"][[0, 2, 4]], st[[1, 3, 5]], rtol=1e-10, atol=1e-12)
    assert np.all(C[[0, 2, 4]][:, [1, 3]] == 0)  # no coupling between the blocks


def refit_sector(seed, n_tracks=300):
    b = synth.sector_workload(seed=seed, n_tracks=n_tracks, truth=True)
    s = b.sector(0)
    o = oracle.track_sector(s["y"], s["z"], s["row"], b.row_x, P, "f32")
    _, sel = oracle.select(len(s["y"]), o["row_hit"], o["n_hits"], o["flags"], P.min_hits)
    out = []
    for t, hits in sel:
        lab = s["label"][hits]
        if np.any(lab != lab[0]) or lab[0] < 0 or len(hits) < 30:
            continue
        r = oracle.fullfit(RX, s["row"][hits], s["y"][hits], s["z"][hits], o["x_ref"][t], o["param"][t],
                           o["first_row"][t], P, "f64")
        if r["flags"] != 1:
            continue
        trk = b.tracks[0]
        L = lab[0]
        last = hits[-1]
        truth = [s["y_true"][last], s["z_true"][last], s["sinphi_true"][last], math.sinh(trk["eta"][L]),
                 trk["q"][L] / trk["pt"][L]]
        out.append((r, np.array(truth)))
    return out


def test_pulls_and_chi2_are_standard_on_smeared_tracks():
    fits = refit_sector(1) + refit_sector(2)
    assert len(fits) > 200
    pulls = np.array([(r["param"] - t) / np.sqrt(np.diag(unpack(r["cov"]))) for r, t in fits])
    mean, rms = pulls.mean(0), np.sqrt((pulls ** 2).mean(0))
    assert np.all(np.abs(mean) < 0.15), mean
    assert np.all((rms > 0.85) & (rms < 1.2)), rms
    chi2ndf = np.array([r["chi2"] / r["ndf"] for r, _ in fits])
    assert 0.85 < chi2ndf.mean() < 1.15


def test_covariances_are_positive_definite():
    for r, _ in refit_sector(3, 200):
        np.linalg.cholesky(unpack(r["cov"]))


def test_bad_input_is_flagged():
    r = oracle.fullfit(RX, np.zeros(0, np.int32), [], [], RX[0], [0, 0, 0, 0, 0], 0, P, "f64")
    assert r["flags"] == 64
    r = oracle.fullfit(RX, np.array([5, 6], np.int32), [0, 0], [0, 0], RX[7], [0, 0, 0, 0, 0], 7, P, "f64")
    assert r["flags"] == 64


@pytest.mark.parametrize("s0,l,q", [(0.3, 0.8, 2.0), (-0.5, -0.4, -3.0), (0.1, 1.2, 0.7)])
def test_transport_jacobian_matches_finite_differences(s0, l, q):
    """The covariance transport C <- F C F^T uses the first-order Jacobian of
    one row step, coupling terms included: a unit variance on one parameter
    shows column j of F in the transported covariance, and it must match the
    finite-difference derivative of the transported state within the
    step's second-order terms."""
    x0, x1 = 150.0, 151.03
    p0 = np.array([4.0, 30.0, s0, l, q])
    h = 1e-6
    for j in (2, 3, 4):
        C = np.zeros(15)
        C[TRI[j, j]] = 1.0
        _, _, C1, rc = oracle.fullfit_transport(x0, p0, C, x1, P)
        assert rc == 0
        Fj = unpack(C1)[:, j]
        e = np.zeros(5)
        e[j] = h
        _, pa, _, _ = oracle.fullfit_transport(x0, p0 + e, np.zeros(15), x1, P)
        _, pb, _, _ = oracle.fullfit_transport(x0, p0 - e, np.zeros(15), x1, P)
        num = (pa - pb) / (2 * h)
        for i in range(5):
            if i == j:
                continue
            assert abs(Fj[i] - num[i]) <= 2e-2 * abs(num[i]) + 1e-9, (i, j, Fj[i], num[i])
