"""Least-squares interpolation (the paper's least-squares interpolation
subsection): a prolongation P whose rows interpolate given prototype vectors
as well as possible in the energy-weighted least-squares sense.

This module is test infrastructure: the CPU oracle against which the GPU
path is checked.

Every fine feature i is interpolated from one coarse feature, the
representative r of its cluster (the aggregations here assign each feature to
one cluster), so row i of P holds one value p_i in column labels[i].  It
minimises sum_k eta_k (v_k(i) - p_i v_k(r))^2 over the prototypes v_k, with
eta_k = <(X^T X + beta I) v_k, v_k>, which gives

    p_i = sum_k eta_k v_k(i) v_k(r) / sum_k eta_k v_k(r)^2.

Readings where the paper leaves a choice:
* the representative of a cluster is its member of lowest index unless the
  caller names one; under leader-follower clustering that member is the
  leader, the coarse feature the paper names for it;
* a cluster whose representative has sum_k eta_k v_k(r)^2 = 0 cannot be
  fitted; its members take p_i = 1 (plain aggregation: the coarse correction
  does not depend on the scale of a column of P, so this is the adjusted
  square-root average for that cluster);
* P^T P is no longer the identity, so the Galerkin coarse matrix is
  P^T X^T X P + lambda P^T P, with P^T P = diag(sum of p_i^2 over each
  cluster).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .operator import apply_A


def representatives(labels: np.ndarray, F_C: int) -> np.ndarray:
    """The member of lowest index of every cluster (int64[F_C])."""
    rep = np.full(F_C, -1, dtype=np.int64)
    for i in range(len(labels) - 1, -1, -1):
        rep[labels[i]] = i
    if np.any(rep < 0):
        raise ValueError("empty cluster")
    return rep


def prototype_energies(X, V: np.ndarray, beta: float) -> np.ndarray:
    """eta_k = <(X^T X + beta I) v_k, v_k> for the columns v_k of V (F x K)."""
    V = np.asarray(V, dtype=np.float64)
    return np.array([float(apply_A(X, beta, V[:, k]) @ V[:, k]) for k in range(V.shape[1])])


def ls_weights(V: np.ndarray, eta: np.ndarray, labels: np.ndarray, F_C: int,
               rep: np.ndarray) -> np.ndarray:
    """p (float64[F]): the least-squares interpolation weight of every
    feature from its cluster's representative."""
    V = np.asarray(V, dtype=np.float64)
    eta = np.asarray(eta, dtype=np.float64)
    p = np.empty(V.shape[0])
    for i in range(V.shape[0]):
        r = rep[labels[i]]
        den = float(np.sum(eta * V[r, :] ** 2))
        p[i] = float(np.sum(eta * V[i, :] * V[r, :])) / den if den != 0.0 else 1.0
    return p


def ls_prolongation(labels: np.ndarray, F_C: int, p: np.ndarray) -> sp.csr_matrix:
    """P(i, labels[i]) = p_i."""
    F = len(labels)
    return sp.csr_matrix((np.asarray(p, dtype=np.float64), (np.arange(F), labels)), shape=(F, F_C))


def galerkin_coarse(X, P, lam: float) -> np.ndarray:
    """A_c = P^T (X^T X + lam I) P, dense."""
    Xc = sp.csr_matrix(X, dtype=np.float64) @ P
    Xc = Xc.toarray() if sp.issparse(Xc) else np.asarray(Xc)
    Pd = P.toarray()
    return Xc.T @ Xc + lam * (Pd.T @ Pd)


def leading_prototypes(X, K: int):
    """The K leading eigenvectors of X^T X (columns of an F x K matrix, unit
    norm) and their eigenvalues, descending: the principal directions of the
    feature space that the paper takes as prototypes (its least-squares
    interpolation subsection).  Plain definition: the dense symmetric
    eigendecomposition of X^T X."""
    G = (sp.csr_matrix(X, dtype=np.float64).T @ sp.csr_matrix(X, dtype=np.float64)).toarray()
    ev, Q = np.linalg.eigh(G)
    order = np.argsort(-ev, kind="stable")[:K]
    return Q[:, order], ev[order]
