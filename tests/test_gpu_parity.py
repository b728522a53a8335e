"""Parity of the HIP path with the oracle (through the C ABI), on the GPU.

Bar: links, start hits, hit-per-row lists, flags, rows and hit counts
bit-exact against the oracle's binary32 mode, and the binary32 state and
covariance bit-exact too (same operation order, correctly rounded float
operations, no contraction on either side).  Fitted parameters are also
checked against the oracle's binary64 refit of the same hits (the strict
bound and its one named exception are in tests/_tolerance.py).
"""
import math

import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection: the first import on a fresh box is slow)

import oracle
import synth
from _harness import compare_sector, gpu_sector, oracle_params, run_gpu
from _tolerance import assert_parameters

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch


def check_batch(batch, params=None, form="batch", sectors=None, **kw):
    from paper_1712_09430_amd import catpc as C
    params = params or C.catpc_default_params()
    tr, hits, out, st, n = run_gpu(batch, params, form, **kw)
    assert st == C.CATPC_OK, C.catpc_last_error()
    links = out.links_numpy()
    trk = out.tracklets_numpy(n)
    bad = []
    for s in (range(batch.n_sectors) if sectors is None else sectors):
        bad += compare_sector(batch, s, gpu_sector(batch, out, links, trk, s), params)
    assert not bad, "\n".join(bad[:20])
    return tr, hits, out, n, links, trk


def test_fp32_rounding_matches_host():
    torch = _torch()
    from paper_1712_09430_amd import catpc as C
    rng = np.random.default_rng(0)
    n = 1 << 20
    a = (rng.standard_normal(n) * np.exp(rng.uniform(-30, 30, n))).astype(np.float32)
    b = (rng.standard_normal(n) * np.exp(rng.uniform(-30, 30, n))).astype(np.float32)
    a[:8] = [0.0, -0.0, 1e-40, -1e-42, 3.4e38, 1.0, 2.0, 0.1]
    b[:8] = [1.0, 3.0, 7e-39, 1e-40, 0.5, 3.0, 3.0, 0.3]
    da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
    do = torch.empty_like(da)
    with np.errstate(all="ignore"):
        want = [a + b, a - b, a * b, a / b, np.sqrt(np.abs(a))]
    for op in range(5):
        src = da if op != 4 else torch.from_numpy(np.abs(a)).cuda()
        C.catpc_fp32_probe(op, src.data_ptr(), db.data_ptr(), do.data_ptr(), n, None)
        torch.cuda.synchronize()
        got = do.cpu().numpy()
        assert np.array_equal(got.view(np.uint32), want[op].astype(np.float32).view(np.uint32)), op


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_one_sector_bit_exact(seed):
    _torch()
    b = synth.sector_workload(seed=seed)
    check_batch(b)


def test_plain_equals_batch_and_oracle():
    _torch()
    b = synth.batch_workload(seed=3, n_events=3, lo=20, hi=600)
    _, _, _, n1, l1, t1 = check_batch(b, form="plain")
    _, _, _, n2, l2, t2 = check_batch(b, form="batch")
    assert n1 == n2
    for k in l1:
        assert np.array_equal(l1[k], l2[k]), k
    for k in t1:
        assert np.array_equal(t1[k], t2[k]), k


def test_small_uneven_batch_bit_exact():
    _torch()
    b = synth.batch_workload(seed=4, n_events=4, lo=20, hi=2000)
    check_batch(b)


@pytest.mark.parametrize("sync", [0, 1])
def test_work_counts_match_oracle_counters(sync):
    """The tracklet kernel's own count of transports, updates, gated
    candidates and row searches equals the oracle's count on the same data,
    whatever the kernel's schedule."""
    _torch()
    b = synth.batch_workload(seed=13, n_events=2, lo=50, hi=1500)
    tr, hits, out, st, n = run_gpu(b, tuning={"tc_sync": sync})
    got = tr.work_counts()
    want = np.zeros(4, np.int64)
    for s in range(b.n_sectors):
        sec = b.sector(s)
        o = oracle.track_sector(sec["y"], sec["z"], sec["row"], b.row_x, oracle.Params(), "f32")
        want += o["counters"]
    assert got.tolist() == want.tolist()


def test_tuning_rejects_block_sizes_beyond_the_kernels():
    from paper_1712_09430_amd import catpc as C
    b = synth.sector_workload(seed=0)
    from paper_1712_09430_amd.tracker import Tracker
    tr = Tracker(b.row_x, 100, 1)
    with pytest.raises(C.CatpcError):
        tr.set_tuning({"nf_block": 1024})
    with pytest.raises(C.CatpcError):
        tr.set_tuning({"tc_block": 512})


def test_parameters_against_f64_refit():
    _torch()
    b = synth.sector_workload(seed=7)
    _, _, out, n, links, trk = check_batch(b)
    s = b.sector(0)
    r = oracle.refit(s["y"], s["z"], b.row_x, trk["row_hit"], trk["start_row"], oracle.Params(), "f64")
    good = (r["flags"] & 1) != 0
    exc = assert_parameters(trk["param"][good], r["param"][good], r["cov"][good], "GPU sector, seed 7")
    print(f"{good.sum()} tracklets, q/pT exceptions (index, sigma, deviation): {exc}")


def test_tuning_does_not_change_results():
    _torch()
    b = synth.batch_workload(seed=5, n_events=2, lo=200, hi=3000)
    _, _, _, n0, l0, t0 = check_batch(b, sectors=[0, 17, 40])
    for tun in ({"bin_hits": 0.5, "nf_block": 64, "tc_block": 64, "tc_waves_per_cu": 1, "use_graph": 0,
                 "nf_rows": 1, "nf_lds_kb": 0, "tc_xcd": 0, "tc_occupancy": 8, "tc_sync": 1},
                {"bin_hits": 16.0, "nf_block": 128, "tc_block": 128, "tc_waves_per_cu": 32, "use_graph": 1,
                 "nf_rows": 16, "nf_lds_kb": 64, "tc_xcd": 1, "tc_occupancy": 8},
                {"bin_hits": 1.0, "nf_block": 256, "tc_block": 256, "tc_waves_per_cu": 3, "use_graph": 1,
                 "nf_rows": 3, "nf_lds_kb": 8, "tc_xcd": 1, "tc_occupancy": 6, "tc_sync": 1},
                {"bin_hits": 0.5, "nf_block": 64, "tc_block": 64, "tc_waves_per_cu": 2, "use_graph": 0,
                 "nf_rows": 2, "nf_lds_kb": 32, "tc_xcd": 0, "tc_occupancy": 6},
                {"bin_hits": 2.0, "nf_block": 256, "tc_block": 256, "tc_waves_per_cu": 8, "use_graph": 1,
                 "nf_rows": 32, "nf_lds_kb": 24, "tc_xcd": 1, "tc_occupancy": 0}):
        _, _, out, st, n = run_gpu(b, tuning=tun)
        assert n == n0
        l1, t1 = out.links_numpy(), out.tracklets_numpy(n)
        for k in l0:
            assert np.array_equal(l0[k], l1[k]), (tun, k)
        for k in t0:
            assert np.array_equal(t0[k], t1[k]), (tun, k)


def test_graph_replays_and_determinism():
    torch = _torch()
    b = synth.batch_workload(seed=6, n_events=2, lo=100, hi=2000)
    tr, hits, out, st, n = run_gpu(b)
    ref_l, ref_t = out.links_numpy(), out.tracklets_numpy(n)
    for rep in range(3):
        out.row_hit.fill_(-7)
        out.param.fill_(float("nan"))
        x = torch.randn(1000, device="cuda").sum()  # unrelated eager work between replays
        tr.track(hits, out)
        st2, n2 = tr.result()
        assert st2 == 0 and n2 == n and torch.isfinite(x)
        l, t = out.links_numpy(), out.tracklets_numpy(n)
        for k in ref_l:
            assert np.array_equal(ref_l[k], l[k]), (rep, k)
        for k in ref_t:
            assert np.array_equal(ref_t[k], t[k]), (rep, k)


def test_capacity_overflow_and_late_fetch():
    _torch()
    from paper_1712_09430_amd import catpc as C
    b = synth.batch_workload(seed=8, n_events=2, lo=100, hi=1000)
    tr, hits, full, st, n = run_gpu(b)
    assert st == C.CATPC_OK and n > 50
    ref = full.tracklets_numpy(n)
    cap = n // 3
    small = tr.output(hits, cap)
    tr.track(hits, small)
    st, n2 = tr.result()
    assert st == C.CATPC_E_CAPACITY and n2 == n
    got = small.tracklets_numpy(cap)
    for k in ref:
        assert np.array_equal(got[k], ref[k][:cap]), k
    rest = tr.output(hits, n - cap)
    tr.fetch(hits, cap, rest)
    tr.result()
    got = rest.tracklets_numpy(n - cap)
    for k in ref:
        assert np.array_equal(got[k], ref[k][cap:]), k


def test_invalid_rows_are_reported():
    _torch()
    from paper_1712_09430_amd import catpc as C
    b = synth.sector_workload(seed=9)
    row = b.row.copy()
    row[100], row[101] = row[101] + 1, row[100]  # break the sort order
    b.row = row
    with pytest.raises(C.CatpcError) as e:
        run_gpu(b)
    assert e.value.status == C.CATPC_E_INVALID
    b2 = synth.sector_workload(seed=9)
    b2.row = b2.row.copy()
    b2.row[-1] = 159
    with pytest.raises(C.CatpcError) as e:
        run_gpu(b2)
    assert e.value.status == C.CATPC_E_INVALID
    # rows fall where each sector starts; a fall inside a later sector of a
    # batch (not at its start) is reported
    b3 = synth.batch_workload(seed=7, n_events=1, lo=20, hi=3000)
    s = 1 + int(np.argmax(np.diff(b3.hit_offset)[1:] > 50))
    assert b3.hit_offset[s + 1] - b3.hit_offset[s] > 50
    j = int(b3.hit_offset[s]) + 40
    b3.row = b3.row.copy()
    b3.row[j], b3.row[j + 1] = b3.row[j + 1] + 1, b3.row[j]
    with pytest.raises(C.CatpcError) as e:
        run_gpu(b3)
    assert e.value.status == C.CATPC_E_INVALID
    # the context stays usable after an invalid input
    check_batch(synth.sector_workload(seed=9))


def row_partition(rows, n_rows):
    """Row of every hit as the row-index pass assigns it: the first hit of each
    row by binary search over the sector (row 0 starts at the sector's first
    hit), as the kernel searches.  Host-side check of a constructed input."""
    n = len(rows)
    first = [0]
    for r in range(1, n_rows):
        lo, hi = 0, n
        while lo < hi:
            mid = (lo + hi) >> 1
            if rows[mid] < r:
                lo = mid + 1
            else:
                hi = mid
        first.append(lo)
    first.append(n)
    part = np.empty(n, np.int64)
    for r in range(n_rows):
        part[first[r]:first[r + 1]] = r
    return part


@pytest.mark.parametrize("dead,p,bad", [(None, 3, -1), (2, 6, 100000)])
def test_out_of_range_row_on_a_start_hit(dead, p, bad):
    """A start hit whose row value is outside the sector's rows: two noise-free
    tracks (two hits per live row); hit p is the start hit of one of them
    (row 1, or row 4 above a dead row 2), and its row is set to `bad` at a
    position where the row-index pass still assigns every hit its own row, so
    that hit still starts a tracklet.  The input is reported invalid, and the
    tracklet kernel writes nothing outside that tracklet's slot: guard records
    on both sides of the hit-per-row output stay untouched, the other
    tracklet equals the oracle's on the valid input, and the bad one records
    nothing."""
    torch = _torch()
    import ctypes

    from paper_1712_09430_amd import catpc as C
    from paper_1712_09430_amd.tracker import DeviceHits, Tracker
    a0 = synth.sector_alpha(0)
    kw = {} if dead is None else {"dead_rows": (dead, 1)}
    b = synth.tracks_workload({"q": [1, -1], "pt": [5.0, 4.0], "eta": [0.2, 0.5], "phi0": [a0 - 0.05, a0 + 0.05]},
                              sigma=0.0, noise_frac=0.0, **kw)
    R = len(b.row_x)
    assert np.array_equal(b.row, np.repeat([r for r in range(R) if r != dead], 2))
    s = b.sector(0)
    ref = oracle.track_sector(s["y"], s["z"], s["row"], b.row_x, oracle.Params(), "f32")
    assert len(ref["start"]) == 2 and p in ref["start"].tolist()
    j = ref["start"].tolist().index(p)
    rows = b.row.copy()
    rows[p] = bad
    assert np.array_equal(row_partition(rows, R), b.row)
    hits = DeviceHits(b.y, b.z, rows, b.hit_offset)
    tr = Tracker(b.row_x, hits.n_hits, 1)
    out = tr.output(hits)
    stride, cap = out.row_stride, out.capacity
    sentinel = -7
    guarded = torch.full(((cap + 2) * stride,), sentinel, dtype=torch.int32, device="cuda:0")
    out.row_hit = guarded[stride:(cap + 1) * stride].view(cap, stride)
    out.struct.row_hit = ctypes.c_void_p(out.row_hit.data_ptr())
    print(f"dead row {dead}, hit {p} row -> {bad}, tracklet slot {j}", flush=True)
    tr.track(hits, out)
    with pytest.raises(C.CatpcError) as e:
        tr.result()
    assert e.value.status == C.CATPC_E_INVALID
    g = guarded.cpu().numpy()
    assert np.all(g[:stride] == sentinel) and np.all(g[(cap + 1) * stride:] == sentinel)
    links = out.links_numpy()
    assert np.array_equal(links["nf_up"], ref["link_up"]) and np.array_equal(links["nf_dn"], ref["link_dn"])
    assert np.array_equal(links["start_hit"], ref["start"])
    trk = out.tracklets_numpy(2)
    assert trk["start_row"][j] == -1 and trk["flags"][j] == 0 and trk["n_hits"][j] == 0
    assert np.all(out.row_hit[j].cpu().numpy() == -1)
    k = 1 - j
    for key in ("row_hit", "start_row", "first_row", "last_row", "n_hits", "flags"):
        assert np.array_equal(trk[key][k], ref[key][k]), key
    for key in ("x_ref", "param", "cov"):
        assert np.array_equal(trk[key][k].view(np.uint32), ref[key][k].view(np.uint32)), key


def test_edge_cases():
    _torch()
    from paper_1712_09430_amd import catpc as C
    # batch with empty sectors, a sector with a single hit, sparse rows
    tracks = {"q": [1.0], "pt": [2.0], "eta": [0.3], "phi0": [math.radians(10.0)]}
    one = synth.tracks_workload(tracks, sigma=0.0, noise_frac=0.0)
    b = synth.batch_workload(seed=10, n_events=1, lo=20, hi=30)  # mostly near-empty sectors
    parts = [(0, 0, {"n_hits": one.n_hits, "hit_offset": np.array([0, 0, one.n_hits, one.n_hits + 1]),
                     "x": np.concatenate([one.x, one.x[:1]]), "y": np.concatenate([one.y, one.y[:1]]),
                     "z": np.concatenate([one.z, one.z[:1]]), "row": np.concatenate([one.row, one.row[:1]]),
                     "label": np.concatenate([one.label, one.label[:1]]), "y_true": None, "tracks": {}})]
    parts[0][2]["n_hits"] = one.n_hits + 1
    e = synth.Batch(parts)
    check_batch(e)
    check_batch(b)
    # nothing at all
    from paper_1712_09430_amd.tracker import DeviceHits, Tracker
    tr = Tracker(b.row_x, 10, 4)
    hits = DeviceHits(np.zeros(0), np.zeros(0), np.zeros(0), np.array([0, 0, 0]))
    out = tr.output(hits, 1)
    tr.track(hits, out)
    st, n = tr.result()
    assert st == C.CATPC_OK and n == 0
    assert out.tracklet_offset.cpu().numpy().tolist() == [0, 0, 0]


def test_precision_form_bit_exact():
    _torch()
    from paper_1712_09430_amd import catpc as C
    b = synth.sector_workload(seed=11)
    for prec in (1, 2):
        p = C.catpc_default_params()
        p.precision = prec
        _, _, _, n, _, trk = check_batch(b, params=p)
        if prec == 2:
            assert np.all(trk["flags"] & C.FLAG_REFIT64)


def _spd64(c):
    """Positive pivots of both covariance blocks in binary64 (packed lower
    triangle: transverse y, sin phi, q/pT; longitudinal z, tan lambda)."""
    t = np.array([[c[0], c[3], c[10]], [c[3], c[5], c[12]], [c[10], c[12], c[14]]], np.float64)
    lo = np.array([[c[2], c[7]], [c[7], c[9]]], np.float64)
    try:
        np.linalg.cholesky(t)
        np.linalg.cholesky(lo)
    except np.linalg.LinAlgError:
        return False
    return True


@pytest.mark.parametrize("sigma", [5e-4, 3e-4])
def test_precision_form_repairs_real_spd_failures(sigma):
    """Precise clusters (smear and fit error sigma cm in both coordinates)
    drive some binary32 covariances to a non-positive pivot: the precision
    form (Sec. 2 item 2; binary32 filter, binary64 covariance only for the
    tracklets that fail the check) refits exactly those, bit for bit as the
    oracle does, and their stored covariances are positive definite."""
    _torch()
    from paper_1712_09430_amd import catpc as C
    b = synth.sector_workload(seed=11, sigma=sigma)
    flags = {}
    for prec in (0, 1):
        p = C.catpc_default_params()
        p.sigma_y = p.sigma_z = sigma
        p.precision = prec
        _, _, _, n, _, trk = check_batch(b, params=p)
        flags[prec] = trk["flags"]
        fail = np.flatnonzero(trk["flags"] & C.FLAG_SPD_FAIL)
        assert len(fail) >= 1
        refit = (trk["flags"] & C.FLAG_REFIT64) != 0
        if prec == 0:
            assert not refit.any()
            assert not any(_spd64(trk["cov"][i]) for i in fail)
        else:
            assert np.array_equal(np.flatnonzero(refit), fail)
            assert all(_spd64(trk["cov"][i]) for i in fail)
    assert np.array_equal(flags[0] & C.FLAG_SPD_FAIL, flags[1] & C.FLAG_SPD_FAIL)


def test_invariants_and_one_hypothesis_per_seed():
    _torch()
    b = synth.event_workload(seed=12, n_tracks=2000)
    from paper_1712_09430_amd import catpc as C
    tr, hits, out, st, n = run_gpu(b)
    links = out.links_numpy()
    up = links["link_up"]
    for s in range(b.n_sectors):
        a, e = int(b.hit_offset[s]), int(b.hit_offset[s + 1])
        u = up[a:e]
        row = b.row[a:e]
        ok = u >= 0
        assert np.all(row[u[ok]] == row[ok] + 1)
        assert len(np.unique(u[ok])) == ok.sum()  # at most one incoming link per hit
    # the hit-per-row record is written in whole 8-row chunks: padding rows hold -1
    rs = C.catpc_row_stride(len(b.row_x))
    assert rs % 8 == 0 and rs >= len(b.row_x) and out.row_hit.shape[1] == rs
    pad = out.row_hit[:n, len(b.row_x):].cpu().numpy()
    assert pad.size == 0 or np.all(pad == -1)


def test_x_input_is_checked_against_the_row_planes():
    _torch()
    from paper_1712_09430_amd import catpc as C
    from paper_1712_09430_amd.tracker import DeviceHits, Tracker
    b = synth.batch_workload(seed=8, n_events=2, lo=100, hi=800)
    assert np.array_equal(b.x, b.row_x[b.row])  # the generator puts hits on the row planes
    tr = Tracker(b.row_x, b.n_hits, b.n_sectors)
    ref = DeviceHits(b.y, b.z, b.row, b.hit_offset)
    out0 = tr.output(ref)
    tr.track(ref, out0)
    st, n = tr.result()
    with_x = DeviceHits(b.y, b.z, b.row, b.hit_offset, x=b.x)
    out1 = tr.output(with_x)
    tr.track(with_x, out1)
    st1, n1 = tr.result()
    assert st == st1 == C.CATPC_OK and n == n1
    assert np.array_equal(out0.tracklets_numpy(n)["param"].view(np.uint32), out1.tracklets_numpy(n)["param"].view(np.uint32))
    bad_x = b.x.copy()
    bad_x[len(bad_x) // 2] += 0.5
    wrong = DeviceHits(b.y, b.z, b.row, b.hit_offset, x=bad_x)
    tr.track(wrong, tr.output(wrong))
    with pytest.raises(C.CatpcError) as e:
        tr.result()
    assert e.value.status == C.CATPC_E_INVALID and "row_x" in str(e.value)
