"""The coarse level (the paper's data-matrices subsection).

P is F x F_C with P(j, s) = 1/sqrt(n_s) when feature j is in cluster s (the
adjusted square-root average interpolation), so P^T P = I.  The Galerkin
coarse matrix is A_c = P^T (X^T X + lam I) P = X_c^T X_c + lam I with
X_c = X P; the coarse system is solved exactly with a Cholesky factor.

Reading: the paper writes the Galerkin product once as P A P^T (in its
two-level iteration subsection) and once as P^T A P (data-matrices
subsection); with P of size F x F_C only P^T A P is defined, so that one is
used throughout.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def cluster_sizes(labels: np.ndarray, F_C: int) -> np.ndarray:
    return np.bincount(labels, minlength=F_C).astype(np.int64)


def prolongation(labels: np.ndarray, F_C: int) -> sp.csr_matrix:
    """P(j, labels[j]) = 1/sqrt(n_{labels[j]})."""
    n = cluster_sizes(labels, F_C)
    F = labels.shape[0]
    vals = 1.0 / np.sqrt(n[labels].astype(np.float64))
    return sp.csr_matrix((vals, (np.arange(F), labels)), shape=(F, F_C))


def averaging_restriction(labels: np.ndarray, F_C: int) -> sp.csr_matrix:
    """The plain averaging restriction P~^T (F_C x F) with entries 1/n_s."""
    n = cluster_sizes(labels, F_C)
    F = labels.shape[0]
    vals = 1.0 / n[labels].astype(np.float64)
    return sp.csr_matrix((vals, (labels, np.arange(F))), shape=(F_C, F))


def _is_binary(X) -> bool:
    data = X.data if sp.issparse(X) else np.asarray(X).ravel()
    return bool(data.size) and bool(np.isin(data, (0.0, 1.0)).all())


def coarse_gram(X, labels: np.ndarray, F_C: int) -> np.ndarray:
    """K = P^T X^T X P = X_c^T X_c (dense F_C x F_C, FP64).

    For 0/1 data X_c = S diag(n)^-1/2 with S = X P_u the integer count
    matrix (P_u the 0/1 membership), so K_st = (S^T S)_st / sqrt(n_s n_t):
    S^T S is formed exactly in integers and scaled once.  Other data use
    FP64 products."""
    if sp.issparse(X) and _is_binary(X):
        n = cluster_sizes(labels, F_C)
        F = labels.shape[0]
        Pu = sp.csr_matrix((np.ones(F, dtype=np.int64), (np.arange(F), labels)), shape=(F, F_C))
        S = sp.csr_matrix(X).astype(np.int64) @ Pu
        StS = np.asarray((S.T @ S).todense(), dtype=np.int64)
        sc = 1.0 / np.sqrt(n.astype(np.float64))
        return (StS.astype(np.float64) * sc[:, None]) * sc[None, :]
    P = prolongation(labels, F_C)
    Xc = X @ P
    K = Xc.T @ Xc
    return np.asarray(K.todense() if sp.issparse(K) else K, dtype=np.float64)


def coarse_matrix(X, labels: np.ndarray, F_C: int, lam: float) -> np.ndarray:
    """A_c = K + lam I (P^T P = I)."""
    return coarse_gram(X, labels, F_C) + lam * np.eye(F_C)


def cholesky(Ac: np.ndarray) -> np.ndarray:
    """Lower-triangular L with L L^T = A_c."""
    return np.linalg.cholesky(Ac)


def coarse_solve(L: np.ndarray, c: np.ndarray) -> np.ndarray:
    """y = A_c^{-1} c via the two triangular solves with L."""
    t = sla.solve_triangular(L, c, lower=True)
    return sla.solve_triangular(L.T, t, lower=False)


def coarse_eigen(K: np.ndarray):
    """(ev, Q) with K = Q diag(ev) Q^T.  The Bayesian-regression experiments
    solve the coarse level with the SVD of X_c (experiments section): its
    right singular vectors and squared singular values are the eigenvectors
    and eigenvalues of K = X_c^T X_c, so the symmetric eigendecomposition
    (LAPACK through NumPy, a library step) stands for it."""
    ev, Q = np.linalg.eigh(np.asarray(K, dtype=np.float64))
    return ev, Q


def eigen_coarse_inverse(ev: np.ndarray, Q: np.ndarray, lam: float) -> np.ndarray:
    """A_c(lam)^-1 = Q diag(1 / (ev + lam)) Q^T: the same decomposition
    serves every lam, with no new factorization."""
    return (Q / (ev + lam)) @ Q.T
