"""Leader-follower clustering of the feature columns of X (the
leader-follower subsection of the paper's clustering section, after
Hartigan), in the form of the paper's experiments: Euclidean distance, and
leaders are not updated when followers join.

This module is test infrastructure: the CPU oracle against which the GPU
path is checked.

The features are visited in their given order.  Each one is compared with
every leader created so far.  If the nearest leader (ties: the one created
first) lies strictly closer than the tolerance, the feature follows it;
otherwise it becomes a new leader.  Cluster s is the s-th leader created.
Reading where the paper leaves a choice: the initial set of clusters is
empty, so feature 0 leads cluster 0.  For 0/1 X the squared distances
c_i + c_s - 2 (X^T X)_{is} are integers, compared with tol^2 exactly.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def leader_follower(X, tol: float):
    """(labels int64[F], F_C, leaders int64[F_C]) for the features of X
    (scipy sparse or dense, N x F) at distance tolerance `tol`.  Small
    problems only: the Gram matrix X^T X is formed densely."""
    Xc = sp.csc_matrix(X, dtype=np.float64)
    G = (Xc.T @ Xc).toarray()
    norms = np.diag(G).copy()
    F = Xc.shape[1]
    tol2 = float(tol) * float(tol)
    labels = np.empty(F, dtype=np.int64)
    leaders: list[int] = []
    for i in range(F):
        if leaders:
            L = np.asarray(leaders)
            d2 = norms[i] + norms[L] - 2.0 * G[i, L]
            s = int(np.argmin(d2))          # first minimum: the earliest leader
            if d2[s] < tol2:
                labels[i] = s
                continue
        labels[i] = len(leaders)
        leaders.append(i)
    return labels, len(leaders), np.asarray(leaders, dtype=np.int64)
