"""Method parameters away from their defaults, each set compared bit for bit
with the oracle through the C ABI: the field (zero: straight tracks, the
helix's degenerate case; reversed; four times stronger, where low-pT tracks
curl out of the sector), windows and cuts narrow, wide and zero, and the miss
limit and hit count at their ends.  Events are generated in the same field as
the one the tracker is given."""
import pytest

import synth
from test_gpu_parity import _torch, check_batch

SETS = {
    "field_zero": dict(bz=0.0),
    "field_reversed": dict(bz=-0.5),
    "field_strong": dict(bz=2.0),
    "narrow": dict(nf_win_y=1.0, nf_win_z=1.0, nf_chi2_max=0.05, tc_gate_nsigma=1.5, tc_max_miss=0, min_hits=3),
    "wide": dict(nf_win_y=6.0, nf_win_z=6.0, nf_chi2_max=2.0, tc_gate_nsigma=6.0, tc_max_miss=10, min_hits=30),
    "zero_cuts": dict(nf_win_y=0.0, nf_win_z=0.0, nf_chi2_max=0.0, tc_gate_nsigma=0.0),
    "asymmetric": dict(nf_win_y=4.0, nf_win_z=1.5, sigma_y=0.05, sigma_z=0.2, tc_max_miss=2),
}


@pytest.mark.gpu
@pytest.mark.parametrize("name", list(SETS))
def test_parameter_sets_match_the_oracle(name):
    _torch()
    from paper_1712_09430_amd import catpc as C
    kv = SETS[name]
    b = synth.sector_workload(seed=21, n_tracks=250, bz=kv.get("bz", synth.BZ))
    p = C.catpc_default_params()
    for k, v in kv.items():
        setattr(p, k, v)
    _, _, _, n, links, trk = check_batch(b, params=p)
    if name == "zero_cuts":
        assert n == 0  # no window admits a second hit of a seed
    else:
        assert n > 0
