"""Sectors with other numbers of pad rows than the TPC's 159 (the library
takes 3 to 4096), compared bit for bit with the oracle through the C ABI, in
the batched and the plain form and under two launch shapes: the row stride of
the hit-per-row records, the 8-row record chunks, the neighbour finder's row
chunks and the tracklet kernel's row planes all follow the row count.  Three
rows leave no room for a seed (a start hit needs an unlinked row below it and
two linked rows above), so that case checks an empty result."""
import math

import pytest

import synth
from test_gpu_parity import _torch, check_batch

A0 = synth.sector_alpha(0)
# (pad rows, tracks of the two events): fewer tracks where the rows are many
CASES = [(3, (150, 40)), (5, (150, 40)), (9, (150, 40)), (17, (150, 40)), (64, (150, 40)), (300, (120, 30)),
         (1000, (60, 20)), (4096, (20, 8))]
SHAPES = [{}, {"nf_rows": 32, "nf_lds_kb": 64, "nf_block": 256, "tc_sync": 1, "tc_block": 64}]


def geometry_batch(n_rows, tracks, **kw):
    """Two events, one A-side sector each, on n_rows planes between the TPC's
    first and last pad-row radii (`kw`: further generator options)."""
    evs = [synth.generate_event(seed, n, i, sectors=(0, 1), n_rows=n_rows, eta=(0.0, 0.9),
                                phi=(A0 - math.radians(10.0), A0 + math.radians(10.0)), **kw)
           for i, (seed, n) in enumerate(zip((11, 12), tracks))]
    b = synth.Batch([(i, 0, ev) for i, ev in enumerate(evs)], n_rows=n_rows)
    assert len(b.row_x) == n_rows and int(b.row.max()) < n_rows
    return b


@pytest.mark.gpu
@pytest.mark.parametrize("n_rows,tracks", CASES)
def test_other_pad_row_counts_match_the_oracle(n_rows, tracks):
    _torch()
    b = geometry_batch(n_rows, tracks)
    for shape in SHAPES:
        *_, n, _, _ = check_batch(b, tuning=shape or None)
        if n_rows == 3:
            assert n == 0
        else:
            assert n > 0
    check_batch(b, form="plain")


@pytest.mark.gpu
@pytest.mark.parametrize("n_rows", [17, 64, 300, 1000])
def test_selection_refit_and_merging_on_other_pad_row_counts(n_rows):
    """The chain after the hot path (tracklet selection, binary64 refit,
    segment merging) on other row counts, against the oracle's own chain; a
    band of 8 dead rows (where the geometry has room for one longer than the
    miss limit) splits tracks into segments for the merging to join."""
    _torch()
    from _harness import run_gpu
    from paper_1712_09430_amd import catpc as C
    from test_gpu_merge import check as check_merges
    from test_gpu_merge import gpu_merges
    from test_gpu_refit import check as check_fits
    dead = (n_rows * 70 // 159, 8) if n_rows >= 64 else (0, 0)
    b = geometry_batch(n_rows, (200, 60) if n_rows < 1000 else (60, 20), dead_rows=dead)
    tr, hits, out, st, n = run_gpu(b)
    assert st == C.CATPC_OK, C.catpc_last_error()
    g, f, m, nt = gpu_merges(tr, hits, out)
    p = C.catpc_default_params()
    sectors = range(b.n_sectors)
    assert nt > 0
    check_fits(b, g, f, p, sectors)
    links = check_merges(b, g, m, p, sectors)
    if dead[1]:
        assert links > 0
