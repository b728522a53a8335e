"""Shared helpers of the GPU tests: run the HIP path through the C ABI and
compare each sector with the oracle on the same seeded input."""
import numpy as np

import oracle
from paper_1712_09430_amd import catpc as C

TRACKLET_KEYS = ("x_ref", "param", "cov", "row_hit", "start_row", "first_row", "last_row", "n_hits", "flags")


def oracle_params(p):
    """oracle.Params with the same values as a catpc_params struct."""
    return oracle.Params(bz=p.bz, sigma_y=p.sigma_y, sigma_z=p.sigma_z, nf_win_y=p.nf_win_y, nf_win_z=p.nf_win_z,
                         nf_chi2_max=p.nf_chi2_max, tc_gate_nsigma=p.tc_gate_nsigma, tc_max_miss=p.tc_max_miss,
                         min_hits=p.min_hits, precision=p.precision)


def run_gpu(batch, params=None, form="batch", capacity=None, tuning=None, tracker=None, device="cuda:0"):
    """Run the hot path on a synth.Batch; returns (tracker, hits, out, status, n_tracklets)."""
    from paper_1712_09430_amd.tracker import DeviceHits, Tracker
    hits = DeviceHits(batch.y, batch.z, batch.row, batch.hit_offset, device)
    if tracker is None:
        tracker = Tracker(batch.row_x, max(hits.n_hits, 1), max(hits.n_sectors, 1), params=params, tuning=tuning,
                          device=device)
    out = tracker.output(hits, capacity)
    tracker.track(hits, out, form)
    st, n = tracker.result()
    return tracker, hits, out, st, n


def gpu_sector(batch, out, links, trk, s):
    """Slice sector s out of GPU results (links dict from out.links_numpy(),
    trk from out.tracklets_numpy(n))."""
    a, b = int(batch.hit_offset[s]), int(batch.hit_offset[s + 1])
    off = links["tracklet_offset"]
    t0, t1 = int(off[s]), int(off[s + 1])
    d = {"nf_up": links["nf_up"][a:b], "nf_dn": links["nf_dn"][a:b], "up_clean": links["link_up"][a:b],
         "dn_clean": links["link_dn"][a:b], "start": links["start_hit"][t0:t1]}
    for k in TRACKLET_KEYS:
        d[k] = trk[k][t0:t1]
    return d


def compare_sector(batch, s, g, params, mode="f32"):
    """Bit-exact comparison of one sector with the oracle; returns a list of
    mismatch descriptions (empty when identical)."""
    sec = batch.sector(s)
    o = oracle.track_sector(sec["y"], sec["z"], sec["row"], batch.row_x, oracle_params(params), mode)
    bad = []
    for gk, ok in (("nf_up", "link_up"), ("nf_dn", "link_dn"), ("up_clean", "up_clean"), ("dn_clean", "dn_clean"),
                   ("start", "start")):
        if not np.array_equal(g[gk], o[ok]):
            idx = np.flatnonzero(g[gk] != o[ok])[:5] if len(g[gk]) == len(o[ok]) else "length"
            bad.append(f"sector {s}: {gk} differs at {idx}")
    if bad:
        return bad
    for k in TRACKLET_KEYS:
        a, b = g[k], o[k]
        if a.shape != b.shape or not np.array_equal(a.view(np.uint8) if a.dtype == np.float32 else a,
                                                    b.view(np.uint8) if b.dtype == np.float32 else b):
            if a.shape == b.shape:
                diff = np.flatnonzero((a != b).reshape(len(a), -1).any(1))[:5]
            else:
                diff = f"shape {a.shape} vs {b.shape}"
            bad.append(f"sector {s}: tracklet field {k} differs at tracklets {diff}")
    return bad


def oracle_merge_sector(batch, s, P, mp=None):
    """The oracle's own chain on sector s (tracklets, selection, binary64
    refit rounded to binary32 as the refit output stores it, merging).
    Returns (next, chi2, labels) with sector-local track indices; labels =
    the most frequent generator label of each track's hits."""
    sec = batch.sector(s)
    o = oracle.track_sector(sec["y"], sec["z"], sec["row"], batch.row_x, P, "f32")
    _, want = oracle.select(len(sec["y"]), o["row_hit"], o["n_hits"], o["flags"], P.min_hits)
    n = len(want)
    ok = np.zeros(n, np.int32)
    a_last = np.zeros(n, np.int32)
    b_first = np.zeros(n, np.int32)
    e_x, s_x = np.zeros(n, np.float32), np.zeros(n, np.float32)
    e_p, s_p = np.zeros((n, 5), np.float32), np.zeros((n, 5), np.float32)
    e_C, s_C = np.zeros((n, 15), np.float32), np.zeros((n, 15), np.float32)
    labels = np.full(n, -1, np.int64)
    for k, (t, hits) in enumerate(want):
        r = oracle.fullfit(batch.row_x, sec["row"][hits], sec["y"][hits], sec["z"][hits], o["x_ref"][t],
                           o["param"][t], o["first_row"][t], P, mode="f64")
        ok[k] = r["flags"] == 1
        a_last[k] = sec["row"][hits[-1]]
        e_x[k], e_p[k], e_C[k] = r["x"], r["param"], r["cov"]
        b_first[k], s_x[k], s_p[k], s_C[k] = o["first_row"][t], o["x_ref"][t], o["param"][t], o["cov"][t]
        if "label" in sec:
            v, c = np.unique(sec["label"][hits], return_counts=True)
            labels[k] = v[np.argmax(c)]
    nxt, chi2 = oracle.merge(batch.row_x, ok, a_last, e_x, e_p, e_C, b_first, s_x, s_p, s_C, P, mp)
    return nxt, chi2, labels


def chains(nxt):
    """prev and head of every segment from the next links (plain walk)."""
    n = len(nxt)
    prev = np.full(n, -1, np.int32)
    for a in range(n):
        if nxt[a] >= 0:
            prev[nxt[a]] = a
    head = np.arange(n, dtype=np.int32)
    for a in range(n):
        while prev[head[a]] >= 0:
            head[a] = prev[head[a]]
    return prev, head
