"""Full Kalman refit of the selected tracks on the GPU against the oracle
(Sec. 2 item 4): the refit runs in binary64 on both sides, so for every
track x, parameters, covariance and chi^2 (stored as binary32) equal the
binary64 oracle's refit of the oracle's own selected track rounded to
binary32, bit for bit, and ndf and flags are equal."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection: the first import on a fresh box is slow)

import oracle
import synth
from _harness import oracle_params, run_gpu

pytestmark = pytest.mark.gpu
FIT_KEYS = ("param", "cov")


def gpu_fits(tr, hits, out):
    tracks = tr.tracks_output(hits, out)
    tr.select(hits, out, tracks)
    nt, nh = tr.select_result()
    fits = tr.fits_output(tracks)
    tr.refit(hits, out, tracks, fits)
    torch.cuda.synchronize()
    return tracks.numpy(nt, nh), fits.numpy(nt), nt


def compare_sector_fits(b, s, g, f, params):
    sec = b.sector(s)
    P = oracle_params(params)
    o = oracle.track_sector(sec["y"], sec["z"], sec["row"], b.row_x, P, "f32")
    _, want = oracle.select(len(sec["y"]), o["row_hit"], o["n_hits"], o["flags"], P.min_hits)
    k0, k1 = int(g["track_offset"][s]), int(g["track_offset"][s + 1])
    if k1 - k0 != len(want):
        return [f"sector {s}: {k1 - k0} tracks, oracle {len(want)}"], []
    bad, d64 = [], []
    for k, (t, hits) in zip(range(k0, k1), want):
        r = oracle.fullfit(b.row_x, sec["row"][hits], sec["y"][hits], sec["z"][hits], o["x_ref"][t],
                           o["param"][t], o["first_row"][t], P, mode="f64")
        for key in ("param", "cov"):
            if not np.array_equal(f[key][k].view(np.uint32), r[key].astype(np.float32).view(np.uint32)):
                bad.append(f"sector {s} track {k}: {key} differs")
        for key in ("x", "chi2"):
            if np.float32(f[key][k]).view(np.uint32) != np.float32(r[key]).view(np.uint32):
                bad.append(f"sector {s} track {k}: {key} differs")
        if f["ndf"][k] != r["ndf"] or f["flags"][k] != r["flags"]:
            bad.append(f"sector {s} track {k}: ndf/flags differ")
        d64.append(r["flags"])
    return bad, d64


def check(b, g, f, params, sectors):
    with ThreadPoolExecutor(max_workers=8) as ex:
        res = list(ex.map(lambda s: compare_sector_fits(b, s, g, f, params), sectors))
    bad = [m for r, _ in res for m in r]
    assert not bad, "\n".join(bad[:20])
    return [x for _, d in res for x in d]


@pytest.mark.parametrize("seed", [1, 2])
def test_one_sector_refit_matches_oracle(seed):
    from paper_1712_09430_amd import catpc as C
    b = synth.sector_workload(seed=seed, n_tracks=300)
    tr, hits, out, st, n = run_gpu(b)
    g, f, nt = gpu_fits(tr, hits, out)
    assert nt > 0 and np.mean(f["flags"] == 1) > 0.95
    flags = check(b, g, f, C.catpc_default_params(), [0])
    assert len(flags) == nt


def test_batch_refit_sampled_sectors_and_properties():
    from paper_1712_09430_amd import autotune
    from paper_1712_09430_amd import catpc as C
    b = synth.batch_workload(seed=3, n_events=8)
    tr, hits, out, st, n = run_gpu(b, tuning=autotune.cached_tuning())
    g, f, nt = gpu_fits(tr, hits, out)
    rng = np.random.default_rng(5)
    sizes = np.diff(b.hit_offset)
    sample = sorted(set(np.argsort(sizes)[-3:].tolist()) | set(rng.choice(b.n_sectors, 12, replace=False).tolist()))
    check(b, g, f, C.catpc_default_params(), sample)
    ok = f["flags"] == 1
    assert ok.mean() > 0.95
    assert np.all(f["ndf"][ok] == 2 * g["track_n_hits"][ok] - 5)
    assert 0.7 < np.mean(f["chi2"][ok] / f["ndf"][ok]) < 1.3


def test_refit_capacity_is_validated():
    from paper_1712_09430_amd import catpc as C
    from paper_1712_09430_amd.tracker import DeviceFits
    b = synth.sector_workload(seed=4, n_tracks=100)
    tr, hits, out, st, n = run_gpu(b)
    tracks = tr.tracks_output(hits, out)
    tr.select(hits, out, tracks)
    tr.select_result()
    small = DeviceFits(max(int(tracks.struct.track_capacity) - 1, 1), "cuda:0")
    with pytest.raises(C.CatpcError) as e:
        tr.refit(hits, out, tracks, small)
    assert e.value.status == C.CATPC_E_INVALID
