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

Reading: the paper recommends CG as the pre-smoother inside flexible CG; a
fixed symmetric smoother keeps B stationary and SPD so the same cycle also
drives plain PCG.
"""
from __future__ import annotations

import numpy as np

from . import coarse as _coarse
from .operator import apply_A, jacobi_diagonal


class TwoLevel:
    def __init__(self, X, lam: float, labels: np.ndarray, F_C: int, omega: float):
        self.X = X
        self.lam = float(lam)
        self.D = jacobi_diagonal(X, lam)
        self.omega = float(omega)
        self.P = _coarse.prolongation(labels, F_C)
        self.Ac = _coarse.coarse_matrix(X, labels, F_C, lam)
        self.L = _coarse.cholesky(self.Ac)

    def smooth(self, r):
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


def make(kind: str, X, lam: float, labels=None, F_C=None, omega=None):
    """Return (apply_B, operator applications per call)."""
    if kind == "none":
        return (lambda r: np.array(r, dtype=np.float64, copy=True)), 0
    D = jacobi_diagonal(X, lam)
    if kind == "jacobi":
        return (lambda r: r / D), 0
    tl = TwoLevel(X, lam, labels, F_C, omega)
    if kind == "vcycle":
        return tl.vcycle, 2
    if kind == "additive":
        return tl.additive, 0
    raise ValueError(kind)
