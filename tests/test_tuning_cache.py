"""The autotuner's cache and the traffic record the bench reads (host logic,
no GPU): the committed cache was tuned on the current kernel source and build
flags, it covers every field of catpc_tuning, it is found only for its own
architecture, the serving tuning is the batch tuning with the serving
search's changes, and the committed traffic record applies to exactly the
cached launch shape (graph replay or not)."""
import json
import os

import bench
from paper_1712_09430_amd import autotune as A
from paper_1712_09430_amd import catpc as C


def cache():
    return json.load(open(A.DEFAULT_CACHE))


def test_cache_was_tuned_on_these_kernels():
    assert A.cache_is_current()
    assert cache()["kernels_sha256"] == bench.kernels_digest()


def test_cache_is_stale_after_a_kernel_change(tmp_path):
    c = cache()
    c["kernels_sha256"] = "0" * 64
    p = tmp_path / "tuning.json"
    p.write_text(json.dumps(c))
    assert not A.cache_is_current(str(p))
    assert not A.cache_is_current(str(tmp_path / "missing.json"))


def test_cache_covers_every_tuning_field():
    fields = {f for f, _ in C.catpc_tuning._fields_}
    assert set(cache()["tuning"]) == fields


def test_cached_tuning_is_found_for_its_architecture_only(tmp_path):
    c = cache()
    arch = c["arch"]
    assert A.cached_tuning(arch) == c["tuning"]
    assert A.cached_tuning(arch.split(":")[0] + ":sramecc-:xnack+") == c["tuning"]  # target features ignored
    assert A.cached_tuning("gfx942") is None
    assert A.cached_tuning(arch, str(tmp_path / "missing.json")) is None


def test_serving_tuning_applies_the_serving_changes():
    c = cache()
    serve = A.cached_serve_tuning(c["arch"])
    assert serve == dict(c["tuning"], **c["serve"]["overrides"])
    assert set(serve) == set(c["tuning"])


def test_traffic_record_applies_to_the_cached_launch_shape_only():
    t = cache()["tuning"]
    rec = bench.profiled_traffic("batch64", t)
    for k in ("k_tracklets", "k_neighbours", "k_grid", "k_clean_start"):
        assert rec[k]["fetch_bytes"] > 0 and rec[k]["write_bytes"] > 0, k
    assert bench.profiled_traffic("batch64", dict(t, use_graph=1 - t["use_graph"])) == rec
    assert bench.profiled_traffic("batch64", dict(t, nf_rows=t["nf_rows"] + 1)) == {}
    assert bench.profiled_traffic("event", t) == {}
    assert os.path.exists(bench.TRAFFIC_PROFILE)
