"""Pins of the leader-follower oracle: the special tolerances, exact
recovery of duplicated columns, and the defining invariants checked by an
independent pure-Python computation on the columns' row sets."""
import numpy as np

import datagen
from oracle import leader


def test_zero_and_huge_tolerance():
    P = datagen.sparse_problem(300, 80, 6, seed=3)
    lab, fc, lead = leader.leader_follower(P.X, 0.0)
    assert fc == 80 and np.array_equal(lab, np.arange(80)) and np.array_equal(lead, np.arange(80))
    lab, fc, lead = leader.leader_follower(P.X, 1e9)
    assert fc == 1 and np.all(lab == 0) and np.array_equal(lead, [0])


def test_duplicated_columns_are_recovered():
    X, groups = datagen.duplicated_columns(400, [3, 1, 5, 2, 4], 0.05, seed=6)
    lab, fc, lead = leader.leader_follower(X, 0.5)   # only identical columns are closer than 0.5
    assert fc == 5
    # every group's first column leads; the group follows it
    for g in range(5):
        members = np.flatnonzero(groups == g)
        assert np.all(lab[members] == lab[members[0]])
        assert lead[lab[members[0]]] == members[0]
    assert len(set(lab[np.flatnonzero(groups == g)][0] for g in range(5))) == 5


def test_invariants_against_row_sets():
    P = datagen.sparse_problem(500, 120, 9, seed=17)
    X = P.X.tocsc()
    rows = [set(X.indices[X.indptr[j]:X.indptr[j + 1]].tolist()) for j in range(120)]
    dist2 = lambda a, b: len(rows[a]) + len(rows[b]) - 2 * len(rows[a] & rows[b])
    for tol in (2.5, 4.0, 5.5):
        lab, fc, lead = leader.leader_follower(X, tol)
        lead = lead.tolist()
        assert lead == sorted(lead) and lab[lead].tolist() == list(range(fc))
        for s, j in enumerate(lead):
            # a leader lies at least tol from every leader created before it
            assert all(dist2(j, lead[t]) >= tol * tol for t in range(s))
        for i in range(120):
            if i in lead:
                continue
            earlier = [t for t in range(fc) if lead[t] < i]
            d = [dist2(i, lead[t]) for t in earlier]
            best = earlier[int(np.argmin(d))]
            assert lab[i] == best and min(d) < tol * tol
