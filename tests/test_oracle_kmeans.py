"""Pins for the oracle's k-means++ over feature columns: brute force with
exact rationals over explicit coordinates, the ideal data set, the objective
invariant and the sampling law of the seeding draws."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

import datagen
from oracle import SplitMix64, kmeans


def _sqdist_frac(a, b):
    return sum((Fraction(x) - Fraction(y)) ** 2 for x, y in zip(a, b))


def _brute_seed(Xd, k, seed):
    """k-means++ seeding from explicit coordinates with exact fractions."""
    F = Xd.shape[1]
    cols = [list(Xd[:, j]) for j in range(F)]
    rng = SplitMix64(seed)
    centres = [rng.next() % F]
    while len(centres) < k:
        d2 = [min(_sqdist_frac(cols[j], cols[c]) for c in centres) for j in range(F)]
        T = sum(d2)
        if T == 0:
            break
        r = rng.next() % int(T)
        acc = 0
        for j in range(F):
            acc += d2[j]
            if acc > r:
                centres.append(j)
                break
    return centres


def _brute_assign(Xd, members):
    """Nearest mean for every feature, exact, ties to the lowest index."""
    F = Xd.shape[1]
    means = {}
    for s, mem in members.items():
        if mem:
            means[s] = [sum(Fraction(Xd[i, j]) for j in mem) / len(mem) for i in range(Xd.shape[0])]
    out = []
    for j in range(F):
        best = None
        for s in sorted(means):
            d = _sqdist_frac(Xd[:, j], means[s])
            if best is None or d < best[0]:
                best = (d, s)
        out.append(best[1])
    return out


@pytest.mark.parametrize("seed", range(6))
def test_seeding_matches_brute_force(seed):
    X = datagen.zipf_binary_csr(12, 8, 3, 1.1, 100 + seed)
    k = 3
    got = list(kmeans.seed_binary(X, k, seed))
    assert got == _brute_seed(X.toarray(), k, seed)


@pytest.mark.parametrize("seed", range(6))
def test_lloyd_matches_brute_force(seed):
    Xd = datagen.zipf_binary_csr(10, 8, 3, 1.1, 200 + seed).toarray()
    k = 2 + seed % 2
    centres = _brute_seed(Xd, k, seed)
    members = {s: [c] for s, c in enumerate(centres)}
    for _ in range(50):
        lab = _brute_assign(Xd, members)
        new = {s: [j for j in range(Xd.shape[1]) if lab[j] == s] for s in range(len(centres))}
        if new == members:
            break
        members = new
    labels, _ = kmeans.lloyd_binary(sp.csr_matrix(Xd), np.array(centres), 100)
    assert list(labels) == _brute_assign(Xd, {s: [j for j in range(Xd.shape[1]) if labels[j] == s]
                                              for s in range(len(centres))})
    assert list(labels) == lab


def test_lloyd_objective_never_increases():
    P = datagen.mid_sparse(n_rows=600, n_cols=200, nnz_per_row=8)
    centres = kmeans.seed_binary(P.X, 12, 3)
    objs = []
    for it in range(1, 8):
        labels, done = kmeans.lloyd_binary(P.X, centres, it)
        objs.append(kmeans.objective(P.X, labels))
        if done < it:
            break
    assert all(b <= a + 1e-9 for a, b in zip(objs, objs[1:]))


def test_fixed_point_at_exit():
    P = datagen.mid_sparse(n_rows=500, n_cols=120, nnz_per_row=6)
    lab, fc, it, _ = kmeans.kmeans_features(P.X, 10, 11)
    assert it < 100
    Xd = P.X.toarray()
    members = {s: list(np.flatnonzero(lab == s)) for s in range(fc)}
    # exact nearest-mean check for a sample of features
    means = {s: Xd[:, m].mean(axis=1) for s, m in members.items()}
    for j in range(0, 120, 7):
        d = [float(((Xd[:, j] - means[s]) ** 2).sum()) for s in range(fc)]
        assert d[lab[j]] <= min(d) + 1e-9


def test_ideal_case_groups_recovered():
    X, group = datagen.duplicated_columns(60, [3, 5, 2, 4, 6], 0.3, seed=4)
    lab, fc, it, _ = kmeans.kmeans_features(X, 5, 17)
    assert fc == 5
    # same partition up to renaming
    pairs = set(zip(group.tolist(), lab.tolist()))
    assert len(pairs) == 5


def test_seeding_distribution():
    """Second centre is drawn with probability D^2_j / T."""
    X = datagen.zipf_binary_csr(30, 6, 3, 0.5, 77)
    Xd = X.toarray()
    c = Xd.sum(axis=0)
    counts = {}
    trials = 3000
    firsts = {}
    for s in range(trials):
        cs = kmeans.seed_binary(X, 2, 1000 + s)
        if len(cs) > 1:
            counts[(cs[0], cs[1])] = counts.get((cs[0], cs[1]), 0) + 1
            firsts[cs[0]] = firsts.get(cs[0], 0) + 1
    for f0, nf in firsts.items():
        if nf < 300:
            continue
        d2 = ((Xd - Xd[:, [f0]]) ** 2).sum(axis=0)
        p = d2 / d2.sum()
        for j in range(6):
            emp = counts.get((f0, j), 0) / nf
            assert abs(emp - p[j]) <= 4 * np.sqrt(p[j] * (1 - p[j]) / nf) + 1e-12


def test_compact_renumbers_in_order():
    lab, fc = kmeans.compact(np.array([4, 4, 1, 7, 1]))
    assert fc == 3 and list(lab) == [1, 1, 0, 2, 0]


def test_real_valued_path_groups():
    Xd = datagen.block_correlated_dense(400, 4, 5, 0.95, seed=3, dtype=np.float64)
    lab, fc, it, _ = kmeans.kmeans_features(Xd, 4, 5, binary=False)
    group = np.repeat(np.arange(4), 5)
    assert len(set(zip(group.tolist(), lab.tolist()))) == fc


# --- real-valued columns -------------------------------------------------------------

def _brute_seed_real(Xd, k, seed):
    """k-means++ seeding on real columns with exact fractions: D^2 to the
    nearest chosen centre, draw r = u T with u = (next() >> 11) / 2^53, the
    next centre the first j whose inclusive prefix of D^2 exceeds r."""
    F = Xd.shape[1]
    cols = [list(Xd[:, j]) for j in range(F)]
    rng = SplitMix64(seed)
    centres = [rng.next() % F]
    while len(centres) < k:
        d2 = [min(_sqdist_frac(cols[j], cols[c]) for c in centres) for j in range(F)]
        T = sum(d2)
        if T == 0:
            break
        r = Fraction(rng.next() >> 11, 1 << 53) * T
        acc = 0
        for j in range(F):
            acc += d2[j]
            if acc > r:
                centres.append(j)
                break
    return centres


@pytest.mark.parametrize("seed", range(6))
def test_real_seeding_matches_brute_force(seed):
    Xd = np.random.default_rng(300 + seed).standard_normal((10, 9))
    assert list(kmeans.seed_real(Xd, 4, seed)) == _brute_seed_real(Xd, 4, seed)


@pytest.mark.parametrize("seed", range(4))
def test_real_lloyd_matches_brute_force(seed):
    """Lloyd from the seeds' member sets, nearest exact mean (ties to the
    lowest index), until no label changes."""
    Xd = np.random.default_rng(400 + seed).standard_normal((8, 14))
    centres = kmeans.seed_real(Xd, 4, seed)
    labels, _ = kmeans.lloyd_real(Xd, centres)
    members = {s: [int(c)] for s, c in enumerate(centres)}
    prev = None
    for _ in range(100):
        new = _brute_assign(Xd, members)
        if new == prev:
            break
        prev = new
        members = {s: [j for j in range(Xd.shape[1]) if new[j] == s] for s in range(len(centres))}
    assert list(labels) == prev


def test_real_seeding_distribution():
    """Real columns: the second centre is drawn with probability D^2_j / T."""
    Xd = np.random.default_rng(78).standard_normal((5, 6)) * np.array([0.5, 1, 1.5, 2, 1, 3])
    trials = 3000
    firsts, counts = {}, {}
    for s in range(trials):
        cs = kmeans.seed_real(Xd, 2, 5000 + s)
        firsts[cs[0]] = firsts.get(cs[0], 0) + 1
        counts[(cs[0], cs[1])] = counts.get((cs[0], cs[1]), 0) + 1
    for f0, nf in firsts.items():
        if nf < 300:
            continue
        d2 = ((Xd - Xd[:, [f0]]) ** 2).sum(axis=0)
        p = d2 / d2.sum()
        for j in range(6):
            emp = counts.get((f0, j), 0) / nf
            assert abs(emp - p[j]) <= 4 * np.sqrt(p[j] * (1 - p[j]) / nf) + 1e-12
