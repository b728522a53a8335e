"""Scheduling baselines (Sec. 3.1: sectors over several queues; Sec. 3.2:
several tracker instances by event): every sector's result equals the
oracle's, bit for bit, whatever queue ran it."""
import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection: the first import on a fresh box is slow)

import synth
from _harness import TRACKLET_KEYS, compare_sector

pytestmark = pytest.mark.gpu


def per_sector(out, n, n_sectors, hit_offset):
    """Each sector's slice of a queue's output, in the form compare_sector takes."""
    links = out.links_numpy()
    trk = out.tracklets_numpy(n)
    toff = links["tracklet_offset"]
    res = []
    for s in range(n_sectors):
        a, b = int(hit_offset[s]), int(hit_offset[s + 1])
        t0, t1 = int(toff[s]), int(toff[s + 1])
        d = {"nf_up": links["nf_up"][a:b], "nf_dn": links["nf_dn"][a:b], "up_clean": links["link_up"][a:b],
             "dn_clean": links["link_dn"][a:b], "start": links["start_hit"][t0:t1]}
        for k in TRACKLET_KEYS:
            d[k] = trk[k][t0:t1]
        res.append(d)
    return res


@pytest.mark.parametrize("q,by,form", [(3, "sector", "plain"), (2, "event", "plain"), (2, "event", "batch")])
def test_queues_match_the_oracle(q, by, form):
    from paper_1712_09430_amd import catpc as C
    from paper_1712_09430_amd.schedule import Queues
    b = synth.batch_workload(seed=4, n_events=3, lo=50, hi=2000)
    Q = Queues(b, q, by=by, form=form)
    Q.run()
    p_def = C.catpc_default_params()
    seen = set()
    bad = []
    for (st_k, n_k), p in zip(Q.check(), Q.parts):
        assert st_k == 0
        got = per_sector(p["out"], n_k, p["hits"].n_sectors, p["hits"].hit_offset_host)
        for j, s in enumerate(p["sectors"]):
            seen.add(s)
            bad += compare_sector(b, s, got[j], p_def)
    assert not bad, "\n".join(bad[:20])
    assert seen == set(range(b.n_sectors))
    assert Q.time_ms(reps=1) > 0
    Q.close()
