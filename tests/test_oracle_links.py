"""Pins for link cleaning and start hits: hand-built link graphs."""
import numpy as np

import oracle


def run(up, dn):
    return oracle.clean_links(np.array(up, np.int32), np.array(dn, np.int32))


def test_mutual_chain_of_five():
    # hits 0..4 in rows 0..4 (one per row), a clean chain 0-1-2-3-4
    up = [-1, 2, 3, 4, -1]
    dn = [-1, 0, 1, 2, -1]
    # hit 0 has no computed links (row 0); 0<-1 is not mutual, so 1 starts
    uc, dc, st = run(up, dn)
    assert uc.tolist() == [-1, 2, 3, -1, -1]
    assert dc.tolist() == [-1, -1, 1, 2, -1]
    assert st.tolist() == [1]


def test_one_sided_links_are_dropped():
    # 1 -> up 2, but 2 points down to 3 (not 1)
    up = [-1, 2, -1, 2, -1]
    dn = [-1, 0, 3, -1, -1]
    uc, dc, st = run(up, dn)
    assert uc.tolist() == [-1, -1, -1, 2, -1]
    assert dc.tolist() == [-1, -1, 3, -1, -1]
    assert st.tolist() == []


def test_chains_of_two_and_three():
    # chain A: 0 <-> 1 (length 2, no start); chain B: 2 <-> 3 <-> 4 (length 3)
    up = [1, -1, 3, 4, -1]
    dn = [-1, 0, -1, 2, 3]
    uc, dc, st = run(up, dn)
    assert uc.tolist() == up and dc.tolist() == dn
    assert st.tolist() == [2]


def test_chains_are_disjoint_paths():
    rng = np.random.default_rng(5)
    n = 400
    up = rng.integers(-1, n, n).astype(np.int32)
    dn = rng.integers(-1, n, n).astype(np.int32)
    for i in range(0, n, 3):  # plant some mutual pairs
        j = (i + 7) % n
        up[i], dn[j] = j, i
    uc, dc, st = run(up, dn)
    # every surviving link is mutual
    for i in range(n):
        if uc[i] >= 0:
            assert dc[uc[i]] == i
        if dc[i] >= 0:
            assert uc[dc[i]] == i
    # at most one incoming surviving up-link per hit
    tgt = uc[uc >= 0]
    assert len(np.unique(tgt)) == len(tgt)
    for s in st:
        assert dc[s] < 0 and uc[s] >= 0 and uc[uc[s]] >= 0
