"""K-means++ over the feature columns of X (the paper's K-means++
subsection of its clustering section; Euclidean distance as in all of the
paper's experiments).

Phase 1, seeding: the first prototype is a feature drawn uniformly; each
further prototype is a feature drawn with probability proportional to its
squared distance to the nearest prototype chosen so far.

Phase 2, Lloyd: assign every feature to its nearest prototype (cluster
mean), recompute the means from the assignment, and repeat until no
assignment changes (or ``max_iter`` assignment passes).

Binary X is handled in exact integer arithmetic so that any other exact
implementation reaches the same labels:

* ||x_j - x_c||^2 = c_j + c_c - 2 (X^T X)_{jc} is an integer;
* a cluster s is held as its member set M_s with S_s = sum_{j in M_s} x_j,
  n_s = |M_s|, Q_s = ||S_s||^2 and G_js = x_j^T S_s (all integers); then
  ||x_j - S_s/n_s||^2 = c_j + (Q_s - 2 n_s G_js) / n_s^2, and the assignment
  compares the rationals (Q_s - 2 n_s G_js) / n_s^2 exactly;
* ties go to the lowest cluster index;
* draws come from SplitMix64: the first centre is next() % F, later ones
  take r = next() % T (T = sum of squared distances) and choose the
  smallest j whose inclusive prefix sum of squared distances exceeds r.
  Seeding stops early if T = 0 (every feature coincides with a centre).

Readings where the paper is silent: the initial member set of cluster s is
its seed {c_s}; a cluster left empty by an assignment is dropped; at the end
the surviving clusters are renumbered in increasing order of their index.

Real-valued X uses the same steps in FP64 (no exactness claim); then the
draw is r = u * T with u = (next() >> 11) * 2^-53.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .splitmix64 import SplitMix64


def _binary_int(X) -> sp.csr_matrix:
    Xi = sp.csr_matrix(X).astype(np.int64)
    if Xi.nnz and not (Xi.data == 1).all():
        raise ValueError("exact mode needs a 0/1 matrix")
    return Xi


def _indicator(labels: np.ndarray, k: int) -> sp.csr_matrix:
    """P_u: the F x k 0/1 membership matrix (rows with label -1 are empty)."""
    F = labels.shape[0]
    rows = np.flatnonzero(labels >= 0)
    return sp.csr_matrix((np.ones(rows.size, dtype=np.int64), (rows, labels[rows])),
                         shape=(F, k))


# --- seeding -----------------------------------------------------------------

def seed_binary(X, k: int, seed: int) -> np.ndarray:
    """k-means++ seeding on the columns of a 0/1 matrix, exact integers.
    Returns the chosen centre features in draw order (fewer than k if T hits
    zero)."""
    Xi = _binary_int(X)
    XT = Xi.T.tocsr()
    F = Xi.shape[1]
    c = np.asarray(Xi.sum(axis=0)).ravel().astype(np.int64)   # ||x_j||^2 (0/1)
    rng = SplitMix64(seed)

    def gram_column(j):
        xj = np.asarray(Xi[:, [j]].todense()).ravel()
        return np.asarray(XT @ xj).ravel().astype(np.int64)

    first = rng.next() % F
    centres = [first]
    d2 = c + c[first] - 2 * gram_column(first)
    while len(centres) < min(k, F):
        T = int(d2.sum())
        if T == 0:
            break
        r = rng.next() % T
        j = int(np.searchsorted(np.cumsum(d2), r, side="right"))
        centres.append(j)
        d2 = np.minimum(d2, c + c[j] - 2 * gram_column(j))
    return np.asarray(centres, dtype=np.int64)


def seed_real(X, k: int, seed: int) -> np.ndarray:
    """k-means++ seeding on real-valued columns in FP64."""
    Xd = X.toarray() if sp.issparse(X) else np.asarray(X, dtype=np.float64)
    F = Xd.shape[1]
    rng = SplitMix64(seed)

    def sqdist_to(j):
        diff = Xd - Xd[:, [j]]
        return np.einsum("ij,ij->j", diff, diff)

    first = rng.next() % F
    centres = [first]
    d2 = sqdist_to(first)
    while len(centres) < min(k, F):
        cs = np.cumsum(d2)
        T = cs[-1]
        if T <= 0:
            break
        r = rng.next_unit() * T
        j = int(np.searchsorted(cs, r, side="right"))
        j = min(j, F - 1)
        centres.append(j)
        d2 = np.minimum(d2, sqdist_to(j))
    return np.asarray(centres, dtype=np.int64)


# --- exact rational argmin ---------------------------------------------------

def exact_argmin(num: np.ndarray, den: np.ndarray, active: np.ndarray) -> np.ndarray:
    """For every row j, the lowest s among active clusters minimizing the
    rational num[j, s] / den[s] (den > 0).  Compares a/b < c/d as
    a*d < c*b in exact integers (Python ints when int64 could overflow)."""
    idx = np.flatnonzero(active)
    bound = int(np.abs(num[:, idx]).max(initial=0)) * int(den[idx].max(initial=1))
    if bound >= (1 << 62):
        num = num.astype(object)
        den = den.astype(object)
    best = np.full(num.shape[0], idx[0], dtype=np.int64)
    bnum = num[:, idx[0]].copy()
    bden = np.full(num.shape[0], den[idx[0]], dtype=num.dtype)
    for s in idx[1:]:
        better = num[:, s] * bden < bnum * den[s]
        best[better] = s
        bnum[better] = num[better, s]
        bden[better] = den[s]
    return best


# --- Lloyd -------------------------------------------------------------------

def lloyd_binary(X, centres: np.ndarray, max_iter: int = 100):
    """Lloyd iterations in exact integers from the member sets {c_s}.
    Returns (labels in 0..k-1 before compaction, number of assignment
    passes)."""
    Xi = _binary_int(X)
    XT = Xi.T.tocsr()
    F = Xi.shape[1]
    k = len(centres)
    labels = np.full(F, -1, dtype=np.int64)
    labels[centres] = np.arange(k)
    it = 0
    while it < max_iter:
        n = np.bincount(labels[labels >= 0], minlength=k).astype(np.int64)
        active = n > 0
        S = (Xi @ _indicator(labels, k)).tocsc()            # N x k counts
        Q = np.asarray(S.multiply(S).sum(axis=0)).ravel().astype(np.int64)
        G = np.asarray((XT @ S).todense(), dtype=np.int64)  # F x k
        num = Q[None, :] - 2 * n[None, :] * G
        den = np.where(active, n * n, 1)
        new = exact_argmin(num, den, active)
        it += 1
        changed = int((new != labels).sum())
        labels = new
        if changed == 0:
            break
    return labels, it


def lloyd_real(X, centres: np.ndarray, max_iter: int = 100):
    """Lloyd iterations in FP64 for real-valued X: score_js =
    ||mu_s||^2 - 2 x_j^T mu_s (the constant ||x_j||^2 dropped), argmin with
    ties to the lowest index."""
    Xd = X.toarray() if sp.issparse(X) else np.asarray(X, dtype=np.float64)
    F = Xd.shape[1]
    k = len(centres)
    labels = np.full(F, -1, dtype=np.int64)
    labels[centres] = np.arange(k)
    it = 0
    while it < max_iter:
        n = np.bincount(labels[labels >= 0], minlength=k).astype(np.float64)
        active = n > 0
        Pu = _indicator(labels, k).toarray().astype(np.float64)
        mu = (Xd @ Pu) / np.where(active, n, 1.0)[None, :]
        score = np.einsum("is,is->s", mu, mu)[None, :] - 2.0 * (Xd.T @ mu)
        score[:, ~active] = np.inf
        new = np.argmin(score, axis=1)   # first minimum = lowest index
        it += 1
        changed = int((new != labels).sum())
        labels = new
        if changed == 0:
            break
    return labels, it


def compact(labels: np.ndarray) -> tuple[np.ndarray, int]:
    """Drop empty clusters and renumber survivors in increasing order."""
    used = np.unique(labels)
    remap = np.full(int(labels.max()) + 1, -1, dtype=np.int64)
    remap[used] = np.arange(used.size)
    return remap[labels].astype(np.int32), int(used.size)


def kmeans_features(X, k: int, seed: int, max_iter: int = 100, binary: bool | None = None):
    """Full k-means++ on the feature columns.  Returns
    (labels int32[F] in 0..F_C-1, F_C, Lloyd passes, centres)."""
    if binary is None:
        data = X.data if sp.issparse(X) else np.asarray(X).ravel()
        binary = bool(data.size) and bool(np.isin(data, (0.0, 1.0)).all())
    if binary:
        centres = seed_binary(X, k, seed)
        labels, it = lloyd_binary(X, centres, max_iter)
    else:
        centres = seed_real(X, k, seed)
        labels, it = lloyd_real(X, centres, max_iter)
    lab, fc = compact(labels)
    return lab, fc, it, centres


def objective(X, labels: np.ndarray) -> float:
    """Within-cluster sum of squared Euclidean distances (FP64)."""
    Xd = X.toarray() if sp.issparse(X) else np.asarray(X, dtype=np.float64)
    tot = 0.0
    for s in np.unique(labels):
        cols = Xd[:, labels == s]
        mu = cols.mean(axis=1, keepdims=True)
        tot += float(((cols - mu) ** 2).sum())
    return tot
