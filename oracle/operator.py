"""The matrix-free operator and the quantities derived from X alone.

The system is the paper's regularized normal equations
(X^T X + lam I) w = X^T y; Krylov methods only need v -> A v (the
introduction: only the matrix-vector product is required, X^T X is never
formed).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .splitmix64 import SplitMix64


def apply_A(X, lam: float, v: np.ndarray) -> np.ndarray:
    """A v = X^T (X v) + lam v in FP64 (two sparse or dense products)."""
    v = np.asarray(v, dtype=np.float64)
    return np.asarray(X.T @ (X @ v), dtype=np.float64) + lam * v


def rhs(X, y: np.ndarray) -> np.ndarray:
    """b = X^T y."""
    return np.asarray(X.T @ np.asarray(y, dtype=np.float64), dtype=np.float64)


def weighted_rows(X, d: np.ndarray):
    """diag(sqrt(d)) X, so that its Gram matrix is X^T D X: the weighted
    operator X^T D X + lam I of Newton steps (the subsection on optimization
    by the Newton method) is apply_A of this matrix, and every coarse-level
    and smoother function of the oracle taken on it is the weighted one.
    Weights d >= 0."""
    d = np.asarray(d, dtype=np.float64)
    if np.any(d < 0) or not np.all(np.isfinite(d)):
        raise ValueError("row weights must be finite and >= 0")
    return sp.diags(np.sqrt(d)) @ (X if sp.issparse(X) else sp.csr_matrix(X))


def noise_rhs(X, y: np.ndarray, tau: float, lam: float, xi1: np.ndarray, xi2: np.ndarray) -> np.ndarray:
    """The right-hand side of one noise-injection sample (Bayesian regression
    subsection, eq. ni_xtx): X^T (y + e1) + e2 / tau with e1 ~ N(0, I_N / tau)
    and e2 ~ N(0, lam I_F), formed from standard-normal draws as
    e1 = xi1 / sqrt(tau), e2 = sqrt(lam) xi2.  The sample solves
    (X^T X + (lam / tau) I) w = this."""
    e1 = np.asarray(xi1, dtype=np.float64) / np.sqrt(tau)
    e2 = np.sqrt(lam) * np.asarray(xi2, dtype=np.float64)
    return rhs(X, np.asarray(y, dtype=np.float64) + e1) + e2 / tau


def column_sq_norms(X) -> np.ndarray:
    """c_j = ||x_j||^2, the diagonal of X^T X."""
    if sp.issparse(X):
        Xc = X.tocsc()
        return np.asarray(Xc.multiply(Xc).sum(axis=0), dtype=np.float64).ravel()
    Xd = np.asarray(X, dtype=np.float64)
    return np.einsum("ij,ij->j", Xd, Xd)


def jacobi_diagonal(X, lam: float) -> np.ndarray:
    """D = diag(A) = ||x_j||^2 + lam (the diagonal preconditioner of DCG)."""
    return column_sq_norms(X) + lam


def is_nonnegative(X) -> bool:
    data = X.data if sp.issparse(X) else np.asarray(X)
    return bool(data.size == 0 or data.min() >= 0)


def gershgorin_row_sums(X) -> np.ndarray:
    """g = X^T (X 1): the row sums of X^T X, which equal its absolute row
    sums when X >= 0 entrywise."""
    ones = np.ones(X.shape[1])
    return np.asarray(X.T @ (X @ ones), dtype=np.float64)


def omega_gershgorin(X, lam: float) -> float:
    """Smoother weight for X >= 0: omega = 1 / rho_hat with
    rho_hat = max_j (g_j + lam) / D_j >= rho(D^-1 A) (Gershgorin's theorem
    applied to the rows of D^-1 A, all of whose entries are >= 0)."""
    if not is_nonnegative(X):
        raise ValueError("Gershgorin weight needs X >= 0; use omega_power")
    g = gershgorin_row_sums(X)
    D = jacobi_diagonal(X, lam)
    return 1.0 / float(np.max((g + lam) / D))


def omega_power(X, lam: float, seed: int, iters: int = 30, safety: float = 1.1) -> float:
    """Smoother weight for general X: omega = 1 / (safety * rho_est), where
    rho_est is the norm ratio after ``iters`` power iterations on
    D^-1/2 A D^-1/2 from a SplitMix64(seed) start vector with entries in
    [0.5, 1.5)."""
    D = jacobi_diagonal(X, lam)
    s = 1.0 / np.sqrt(D)
    rng = SplitMix64(seed)
    v = np.array([rng.next_unit() + 0.5 for _ in range(X.shape[1])])
    v /= np.linalg.norm(v)
    rho = 0.0
    for _ in range(iters):
        w = s * apply_A(X, lam, s * v)
        rho = float(np.linalg.norm(w))
        v = w / rho
    return 1.0 / (safety * rho)


# --- BF16 operands (the correction operator of iterative refinement) -----------

def bf16_round(a) -> np.ndarray:
    """Values rounded to BF16 (8 significant bits), returned as FP64: first
    FP64 -> FP32, then FP32 -> BF16, each to nearest with ties to even.
    BF16 keeps the FP32 exponent, so the second step clears the low 16 bits
    of the FP32 pattern after adding half of their unit (plus the kept
    lowest bit for ties)."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    finite = np.isfinite(f)
    keep = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + keep) >> np.uint64(16)) << np.uint64(16)
    r = np.where(finite, r, u & np.uint64(0xFFFF0000))
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def apply_A_bf16(X, lam: float, V: np.ndarray) -> np.ndarray:
    """The BF16-operand operator on columns V (F x m): X and V rounded to
    BF16, U = X V rounded to BF16, then X^T U + lam V with exact (FP64)
    sums.  This is the definition; a GPU summing in FP32 differs from it by
    at most the rounding of those sums (see apply_A_bf16_bound)."""
    Xb = bf16_round(X.toarray() if sp.issparse(X) else X)
    V = np.asarray(V, dtype=np.float64)
    U = bf16_round(Xb @ bf16_round(V))
    return Xb.T @ U + lam * V


def apply_A_bf16_bound(X, V: np.ndarray) -> np.ndarray:
    """Elementwise bound on |Q - apply_A_bf16(X, lam, V)| for a Q whose two
    products sum exact BF16 x BF16 products in FP32, in any order.  With
    S = |X~| |V~| and gamma_n = n 2^-24 / (1 - n 2^-24): the FP32 sum for U
    errs by at most gamma_F S, so its BF16 rounding differs from that of the
    exact U by at most du = 2^-7 S + 2 gamma_F S; the second sum adds at most
    gamma_N |X~|^T (S + du)."""
    Xb = np.abs(bf16_round(X.toarray() if sp.issparse(X) else X))
    Vb = np.abs(bf16_round(V))
    N, F = Xb.shape

    def gamma(n):
        e = n * 2.0 ** -24
        return e / (1.0 - e)

    S = Xb @ Vb
    du = 2.0 ** -7 * S + 2.0 * gamma(F) * S
    return Xb.T @ du + gamma(N) * (Xb.T @ (S + du))


def f32_round(a) -> np.ndarray:
    """Values rounded to FP32 (nearest, ties to even), returned as FP64."""
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def apply_A_f32(X, lam: float, V: np.ndarray) -> np.ndarray:
    """The FP32-operand operator on columns V (F x m): V rounded to FP32, U =
    X V rounded to FP32, then X^T U + lam V with exact sums (X is FP32
    already).  A GPU summing in FP32 differs by at most apply_A_f32_bound."""
    Xd = f32_round(X.toarray() if sp.issparse(X) else X)
    V = np.asarray(V, dtype=np.float64)
    U = f32_round(Xd @ f32_round(V))
    return Xd.T @ U + lam * V


def apply_A_f32_bound(X, V: np.ndarray) -> np.ndarray:
    """Elementwise bound on |Q - apply_A_f32(X, lam, V)| for FP32 sums in any
    order: with S = |X| |V~|, the computed U differs from the rounded exact
    one by at most du = (gamma_F + 2^-24) S (the sum's error plus one
    rounding), and the second sum adds at most gamma_N |X|^T (S + du)."""
    Xa = np.abs(f32_round(X.toarray() if sp.issparse(X) else X))
    Va = np.abs(f32_round(V))
    N, F = Xa.shape

    def gamma(n):
        e = n * 2.0 ** -24
        return e / (1.0 - e)

    S = Xa @ Va
    du = (gamma(F) + 2.0 ** -24) * S
    return Xa.T @ du + gamma(N) * (Xa.T @ (S + du))
