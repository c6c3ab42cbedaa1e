"""Preconditioners z = B r used inside (P)CG.

* ``none``: z = r (plain CG).
* ``jacobi``: z = D^-1 r with D = diag(A) (the paper's DCG).
* ``vcycle``: the two-level cycle of the paper's two-level iteration
  subsection, whose error propagation is
  T = (I - S A)(I - P A_c^-1 P^T A)(I - S A), here with the Richardson step
  scaled by the Jacobi diagonal, S = omega D^-1 (one pre- and one
  post-smoothing step).  Applied to r with zero initial guess:
      e1 = S r;  rho1 = r - A e1;  e2 = e1 + P A_c^-1 P^T rho1;
      rho2 = r - A e2;  z = e2 + S rho2.
  With omega * rho(D^-1 A) < 2 this B is symmetric positive definite, so
  plain PCG applies.
* ``additive``: z = S r + P A_c^-1 P^T r (no extra operator application).

* ``rougher``: the configuration of the paper's experiments (TLFCG): a
  few iterations of plain CG on A e = r from e = 0 as pre-smoother (the
  paper calls CG a rougher; a Jacobi-preconditioned CG variant is offered
  too), then the coarse correction of the rougher's residual, no
  post-smoothing:
      e1 = CG_s(A, r);  rho = r - A e1 (the CG recurrence residual);
      z = e1 + P A_c^-1 P^T rho.
  It is not a fixed linear map of r, so it drives flexible CG.

Block smoother (the cluster-aligned block option): S = omega D_B^-1 with D_B
the block diagonal of A over blocks that never cross a cluster: each
cluster's members in increasing feature index, cut into consecutive groups
of at most 32.  Its weight comes from the power estimate of rho(D_B^-1 A)
(block_omega).

Reading: the paper recommends CG as the pre-smoother inside flexible CG; a
fixed symmetric smoother keeps B stationary and SPD so the same cycle also
drives plain PCG.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import coarse as _coarse
from . import interp as _interp
from .operator import apply_A, jacobi_diagonal


def smoother_blocks(labels: np.ndarray, F_C: int, size: int = 32) -> list:
    """Feature index arrays of the block smoother: for every cluster in
    order, its members in increasing index cut into groups of <= size."""
    out = []
    for s in range(F_C):
        members = np.flatnonzero(labels == s)
        for a in range(0, members.size, size):
            out.append(members[a:a + size])
    return out


def block_inverses(X, lam: float, blocks: list) -> list:
    """(A_BB)^-1 for every block B, A_BB = X_B^T X_B + lam I (dense FP64)."""
    import scipy.sparse as sp
    Xc = X.tocsc() if sp.issparse(X) else np.asarray(X, dtype=np.float64)
    inv = []
    for B in blocks:
        XB = Xc[:, B]
        XB = XB.toarray() if sp.issparse(XB) else XB
        G = XB.T @ XB + lam * np.eye(B.size)
        inv.append(np.linalg.inv(G))
    return inv


def block_apply(blocks: list, inv: list, r: np.ndarray) -> np.ndarray:
    """D_B^-1 r."""
    z = np.zeros_like(np.asarray(r, dtype=np.float64))
    for B, Gi in zip(blocks, inv):
        z[B] = Gi @ r[B]
    return z


def block_omega(X, lam: float, blocks: list, inv: list, seed: int, iters: int = 30,
                safety: float = 1.1) -> float:
    """omega = 1 / (safety * rho_est), rho_est the norm ratio after `iters`
    power steps v <- D_B^-1 A v / ||.|| (D_B^-1 A is similar to the SPD
    D_B^-1/2 A D_B^-1/2, so its eigenvalues are real and positive) from the
    unit-normalised SplitMix64(seed) start vector with entries in [0.5, 1.5)
    (the same start as operator.omega_power)."""
    from .splitmix64 import SplitMix64
    rng = SplitMix64(seed)
    v = np.array([rng.next_unit() + 0.5 for _ in range(X.shape[1])])
    v /= np.linalg.norm(v)
    rho = 0.0
    for _ in range(iters):
        w = block_apply(blocks, inv, apply_A(X, lam, v))
        rho = float(np.linalg.norm(w))
        v = w / rho
    return 1.0 / (safety * rho)


def cg_rougher(apply_A, r: np.ndarray, steps: int = 2, D=None):
    """`steps` iterations of CG on A e = r from e = 0 (plain CG, or
    Jacobi-preconditioned CG with diagonal D): returns e and the recurrence
    residual r - A e (exact arithmetic).  Stops early when the residual
    vanishes."""
    r = np.asarray(r, dtype=np.float64)
    e = np.zeros_like(r)
    res = r.copy()
    z = res / D if D is not None else res.copy()
    p = z.copy()
    rz = float(res @ z)
    for i in range(steps):
        if rz == 0.0:
            break
        q = apply_A(p)
        alpha = rz / float(p @ q)
        e += alpha * p
        res -= alpha * q
        z = res / D if D is not None else res
        rz_new = float(res @ z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return e, res


class TwoLevel:
    def __init__(self, X, lam: float, labels: np.ndarray, F_C: int, omega: float,
                 smoother: str = "point", block_size: int = 32, P=None):
        self.X = X
        self.lam = float(lam)
        self.D = jacobi_diagonal(X, lam)
        self.omega = float(omega)
        if P is None:       # the adjusted square-root average
            self.P = _coarse.prolongation(labels, F_C)
            self.Ac = _coarse.coarse_matrix(X, labels, F_C, lam)
        else:               # any given prolongation (least-squares interpolation)
            self.P = sp.csr_matrix(P)
            self.Ac = _interp.galerkin_coarse(X, self.P, lam)
        self.L = _coarse.cholesky(self.Ac)
        self.smoother = smoother
        if smoother == "block":
            self.blocks = smoother_blocks(labels, F_C, block_size)
            self.inv = block_inverses(X, lam, self.blocks)

    def smooth(self, r):
        if self.smoother == "block":
            return self.omega * block_apply(self.blocks, self.inv, r)
        return self.omega * r / self.D

    def coarse_correction(self, r):
        c = self.P.T @ r
        return self.P @ _coarse.coarse_solve(self.L, c)

    def vcycle(self, r):
        e1 = self.smooth(r)
        rho1 = r - apply_A(self.X, self.lam, e1)
        e2 = e1 + self.coarse_correction(rho1)
        rho2 = r - apply_A(self.X, self.lam, e2)
        return e2 + self.smooth(rho2)

    def additive(self, r):
        return self.smooth(r) + self.coarse_correction(r)

    def rougher(self, r, steps: int = 2, jacobi: bool = False):
        e1, rho = cg_rougher(lambda v: apply_A(self.X, self.lam, v), r, steps,
                             self.D if jacobi else None)
        return e1 + self.coarse_correction(rho)


def make(kind: str, X, lam: float, labels=None, F_C=None, omega=None, smoother="point", P=None):
    """Return (apply_B, operator applications per call)."""
    if kind == "none":
        return (lambda r: np.array(r, dtype=np.float64, copy=True)), 0
    D = jacobi_diagonal(X, lam)
    if kind == "jacobi":
        return (lambda r: r / D), 0
    tl = TwoLevel(X, lam, labels, F_C, omega, smoother, P=P)
    if kind == "vcycle":
        return tl.vcycle, 2
    if kind == "additive":
        return tl.additive, 0
    if kind == "rougher":
        return tl.rougher, 2
    raise ValueError(kind)
