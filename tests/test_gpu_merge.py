"""Merging of track segments inside a sector on the GPU against the oracle
(Sec. 2 item 3).  The GPU chain (tracklets, selection, binary64 refit,
merging) and the oracle's own chain run on the same seeded events with a
band of dead pad rows, which splits tracks into two segments; per sector the
links (next), their chi^2 (binary32, bit for bit), prev and head equal the
oracle's, and over every sector the links form valid chains."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection: the first import on a fresh box is slow)

import oracle
import synth
from _harness import chains, oracle_merge_sector, oracle_params, run_gpu

pytestmark = pytest.mark.gpu
DEAD = (70, 8)


def gpu_merges(tr, hits, out, cuts=None):
    tracks = tr.tracks_output(hits, out)
    tr.select(hits, out, tracks)
    nt, nh = tr.select_result()
    fits = tr.fits_output(tracks)
    tr.refit(hits, out, tracks, fits)
    merges = tr.merges_output(tracks)
    tr.merge(hits, out, tracks, fits, merges, cuts)
    torch.cuda.synchronize()
    return tracks.numpy(nt, nh), fits.numpy(nt), merges.numpy(nt), nt


def compare_sector_merges(b, s, g, m, params, mp=None):
    P = oracle_params(params)
    nxt, chi2, _ = oracle_merge_sector(b, s, P, mp)
    k0, k1 = int(g["track_offset"][s]), int(g["track_offset"][s + 1])
    if k1 - k0 != len(nxt):
        return [f"sector {s}: {k1 - k0} tracks, oracle {len(nxt)}"], 0
    prev, head = chains(nxt)
    want = {"next": np.where(nxt >= 0, nxt + k0, -1), "prev": np.where(prev >= 0, prev + k0, -1), "head": head + k0}
    bad = []
    for key, w in want.items():
        if not np.array_equal(m[key][k0:k1], w):
            bad.append(f"sector {s}: {key} differs at {np.flatnonzero(m[key][k0:k1] != w)[:5]}")
    if not np.array_equal(m["chi2"][k0:k1].view(np.uint32), chi2.view(np.uint32)):
        bad.append(f"sector {s}: chi2 differs at {np.flatnonzero(m['chi2'][k0:k1] != chi2)[:5]}")
    return bad, int(np.sum(nxt >= 0))


def check(b, g, m, params, sectors, mp=None):
    with ThreadPoolExecutor(max_workers=8) as ex:
        res = list(ex.map(lambda s: compare_sector_merges(b, s, g, m, params, mp), sectors))
    bad = [x for r, _ in res for x in r]
    assert not bad, "\n".join(bad[:20])
    return sum(k for _, k in res)


def check_chains(g, m, nt, cut=25.0):
    nxt, prev, head, chi2 = m["next"], m["prev"], m["head"], m["chi2"]
    sec = np.repeat(np.arange(len(g["track_offset"]) - 1), np.diff(g["track_offset"]))
    a = np.flatnonzero(nxt >= 0)
    assert np.all(prev[nxt[a]] == a) and np.all(sec[nxt[a]] == sec[a])
    assert np.sum(prev >= 0) == len(a)
    assert np.all((chi2 >= 0) == (nxt >= 0)) and np.all(chi2[a] <= cut)
    assert np.all(head[head] == head) and np.all(prev[head] == -1)
    assert np.all(head[nxt[a]] == head[a])
    return len(a)


@pytest.mark.parametrize("seed", [1, 2])
def test_one_sector_merges_match_oracle(seed):
    from paper_1712_09430_amd import catpc as C
    b = synth.sector_workload(seed=seed, n_tracks=300, dead_rows=DEAD)
    tr, hits, out, st, n = run_gpu(b)
    g, f, m, nt = gpu_merges(tr, hits, out)
    links = check(b, g, m, C.catpc_default_params(), [0])
    assert links > 100
    assert check_chains(g, m, nt) == links


def test_batch_merges_sampled_sectors_and_chains():
    from paper_1712_09430_amd import autotune
    from paper_1712_09430_amd import catpc as C
    b = synth.batch_workload(seed=3, n_events=8, dead_rows=DEAD)
    tr, hits, out, st, n = run_gpu(b, tuning=autotune.cached_tuning())
    g, f, m, nt = gpu_merges(tr, hits, out)
    rng = np.random.default_rng(6)
    sizes = np.diff(b.hit_offset)
    sample = sorted(set(np.argsort(sizes)[-3:].tolist()) | set(rng.choice(b.n_sectors, 12, replace=False).tolist()))
    assert check(b, g, m, C.catpc_default_params(), sample) > 0
    assert check_chains(g, m, nt) > 0.2 * nt


@pytest.mark.parametrize("cuts", [(3, 10.0, 25.0), (30, 2.0, 25.0), (30, 10.0, 4.0), (30, 1e6, 1e9)])
def test_cuts_match_oracle(cuts):
    from paper_1712_09430_amd import catpc as C
    b = synth.sector_workload(seed=5, n_tracks=300, dead_rows=DEAD)
    tr, hits, out, st, n = run_gpu(b)
    mp = C.catpc_merge_params(*cuts)
    g, f, m, nt = gpu_merges(tr, hits, out, mp)
    check(b, g, m, C.catpc_default_params(), [0], oracle.MergeParams(*cuts))
    check_chains(g, m, nt, cuts[2])


@pytest.mark.parametrize("cap", [1, 37, 150])
def test_pair_list_overflow_gives_the_same_links(cap):
    """A short candidate-pair list (tuning merge_pair_cap): the tracks whose
    pairs did not fit evaluate them in their own lane; links unchanged."""
    from paper_1712_09430_amd import catpc as C
    b = synth.sector_workload(seed=1, n_tracks=300, dead_rows=DEAD)
    tr, hits, out, st, n = run_gpu(b, tuning={"merge_pair_cap": cap})
    g, f, m, nt = gpu_merges(tr, hits, out)
    assert check(b, g, m, C.catpc_default_params(), [0]) > 100


def test_work_counts_match_the_candidate_tests():
    """catpc_merge_counts: the candidate pairs are those passing the row and
    straight-line window tests (counted here on the GPU's own fit and
    tracklet outputs, in binary64 with the same expressions), and the row
    steps are the rows between the pairs' ends."""
    b = synth.sector_workload(seed=2, n_tracks=300, dead_rows=DEAD)
    tr, hits, out, st, n = run_gpu(b)
    g, f, m, nt = gpu_merges(tr, hits, out)
    pairs, steps = tr.merge_counts()
    trk = out.tracklets_numpy(n)
    slot = g["track_tracklet"][:nt].astype(np.int64)
    last = np.array([b.row[g["track_hits"][g["track_hit_offset"][k] + g["track_n_hits"][k] - 1]]
                     for k in range(nt)])
    first = trk["first_row"][slot]
    sx, sy, sz = (trk["x_ref"][slot].astype(np.float64), trk["param"][slot, 0].astype(np.float64),
                  trk["param"][slot, 1].astype(np.float64))
    ok = f["flags"] == 1
    want_pairs = want_steps = 0
    for a in np.flatnonzero(ok):
        p = f["param"][a].astype(np.float64)
        c = np.sqrt(1.0 - p[2] * p[2])
        ty, tz = p[2] / c, p[3] / c
        for bb in np.flatnonzero(ok):
            if bb == a or not (last[a] < first[bb] <= last[a] + 30):
                continue
            dx0 = sx[bb] - np.float64(f["x"][a])
            if abs((p[0] + dx0 * ty) - sy[bb]) <= 10.0 and abs((p[1] + dx0 * tz) - sz[bb]) <= 10.0:
                want_pairs += 1
                want_steps += int(first[bb] - last[a])
    assert pairs == want_pairs and pairs > 0
    assert 0.9 * want_steps <= steps <= want_steps


def test_no_dead_band_and_empty_sectors():
    from paper_1712_09430_amd import catpc as C
    b = synth.event_workload(seed=2, n_tracks=300)
    tr, hits, out, st, n = run_gpu(b)
    g, f, m, nt = gpu_merges(tr, hits, out)
    check(b, g, m, C.catpc_default_params(), range(b.n_sectors))
    check_chains(g, m, nt)


def test_merge_arguments_are_validated():
    from paper_1712_09430_amd import catpc as C
    from paper_1712_09430_amd.tracker import DeviceMerges
    b = synth.sector_workload(seed=4, n_tracks=100, dead_rows=DEAD)
    tr, hits, out, st, n = run_gpu(b)
    tracks = tr.tracks_output(hits, out)
    tr.select(hits, out, tracks)
    tr.select_result()
    fits = tr.fits_output(tracks)
    tr.refit(hits, out, tracks, fits)
    small = DeviceMerges(max(int(tracks.struct.track_capacity) - 1, 1), "cuda:0")
    with pytest.raises(C.CatpcError) as e:
        tr.merge(hits, out, tracks, fits, small)
    assert e.value.status == C.CATPC_E_INVALID
    merges = tr.merges_output(tracks)
    for bad in [(0, 10.0, 25.0), (5000, 10.0, 25.0), (30, -1.0, 25.0), (30, 10.0, float("nan"))]:
        with pytest.raises(C.CatpcError) as e:
            tr.merge(hits, out, tracks, fits, merges, C.catpc_merge_params(*bad))
        assert e.value.status == C.CATPC_E_INVALID
