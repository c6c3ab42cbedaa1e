"""Krylov solvers for A x = b.

PCG: x_0 = 0 and r_0 = b (the initialisation of the paper's flexible CG
algorithm), stopping when ||r_k|| <= tol ||b|| (the relative residual the
paper plots).  The iteration count is the number of x-updates.

FCG(m): the paper's flexible CG algorithm (after Notay), z_i = M_i^-1 r_i,
p_i = z_i - sum_{k=i-m_i}^{i-1} <z_i, A p_k>/<p_k, A p_k> p_k,
alpha_i = <p_i, r_i>/<p_i, A p_i>, with the truncation m_0 = 0,
m_i = max(1, i mod (m+1)).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

OK, NOT_CONVERGED, BREAKDOWN = 0, 4, 5


@dataclass
class Info:
    status: int
    iters: int
    relres: float
    true_relres: float
    history: list = field(default_factory=list)
    err_history: list = field(default_factory=list)


def pcg(apply_A, b, apply_B, tol=1e-10, max_iter=10_000, fixed_iters=None,
        x_ref=None):
    """Preconditioned CG.  With ``fixed_iters`` exactly that many iterations
    run regardless of the residual.  With ``x_ref`` the relative error of
    every iterate against it is recorded."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return x, Info(OK, 0, 0.0, 0.0)
    r = b.copy()
    z = apply_B(r)
    rz = float(r @ z)
    p = z.copy()
    k = 0
    hist = [1.0]
    errs = []
    refn = float(np.linalg.norm(x_ref)) if x_ref is not None else None
    if x_ref is not None:
        errs.append(1.0)
    status = NOT_CONVERGED
    if not rz > 0:
        return x, Info(BREAKDOWN, 0, 1.0, 1.0, hist)
    limit = fixed_iters if fixed_iters is not None else max_iter
    while k < limit:
        q = apply_A(p)
        pq = float(p @ q)
        if not pq > 0:
            status = BREAKDOWN
            break
        alpha = rz / pq
        x += alpha * p
        r -= alpha * q
        k += 1
        rn = float(np.linalg.norm(r))
        hist.append(rn / bnorm)
        if x_ref is not None:
            errs.append(float(np.linalg.norm(x - x_ref)) / refn)
        if fixed_iters is None and rn <= tol * bnorm:
            status = OK
            break
        z = apply_B(r)
        rz_new = float(r @ z)
        if not rz_new > 0:
            status = BREAKDOWN
            break
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    if fixed_iters is not None and status != BREAKDOWN:
        status = OK
    true = float(np.linalg.norm(b - apply_A(x))) / bnorm
    return x, Info(status, k, hist[-1], true, hist, errs)


def fcg(apply_A, b, apply_B, m=1, tol=1e-10, max_iter=10_000, fixed_iters=None):
    """Flexible CG with truncation parameter m.  ``apply_B(r, i)`` may
    depend on the iteration index i (a variable preconditioner)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    bnorm = float(np.linalg.norm(b))
    if bnorm == 0.0:
        return x, Info(OK, 0, 0.0, 0.0)
    r = b.copy()
    ps, aps, paps = [], [], []
    hist = [1.0]
    status = NOT_CONVERGED
    limit = fixed_iters if fixed_iters is not None else max_iter
    i = 0
    while i < limit:
        z = apply_B(r, i)
        m_i = 0 if i == 0 else max(1, i % (m + 1))
        p = z.copy()
        for kk in range(i - m_i, i):
            p -= (float(z @ aps[kk]) / paps[kk]) * ps[kk]
        q = apply_A(p)
        pq = float(p @ q)
        if not pq > 0:
            status = BREAKDOWN
            break
        alpha = float(p @ r) / pq
        x += alpha * p
        r -= alpha * q
        ps.append(p)
        aps.append(q)
        paps.append(pq)
        i += 1
        rn = float(np.linalg.norm(r))
        hist.append(rn / bnorm)
        if fixed_iters is None and rn <= tol * bnorm:
            status = OK
            break
    if fixed_iters is not None and status != BREAKDOWN:
        status = OK
    true = float(np.linalg.norm(b - apply_A(x))) / bnorm
    return x, Info(status, i, hist[-1], true, hist)


def solve(X, y, lam, method="vcycle", labels=None, F_C=None, omega=None,
          tol=1e-10, max_iter=10_000, fixed_iters=None, x_ref=None, rhs_is_b=False,
          smoother="point", P=None):
    """Convenience wrapper: b = X^T y (or y itself with ``rhs_is_b``), then
    PCG with the named preconditioner (point or block smoother; P replaces
    the adjusted square-root average prolongation when given)."""
    from . import operator as op
    from . import precond
    b = np.asarray(y, dtype=np.float64) if rhs_is_b else op.rhs(X, y)
    if method in ("vcycle", "additive") and omega is None:
        if smoother == "block":
            blocks = precond.smoother_blocks(labels, F_C)
            omega = precond.block_omega(X, lam, blocks, precond.block_inverses(X, lam, blocks), 0x5eed)
        else:
            omega = op.omega_gershgorin(X, lam)
    B, _ = precond.make(method, X, lam, labels, F_C, omega, smoother, P=P)
    return pcg(lambda v: op.apply_A(X, lam, v), b, B, tol, max_iter, fixed_iters, x_ref)


def reference_solution(X, y, lam, rhs_is_b=False):
    """w* = (X^T X + lam I)^-1 b by a dense Cholesky solve (small F)."""
    import scipy.linalg as sla
    from . import operator as op
    b = np.asarray(y, dtype=np.float64) if rhs_is_b else op.rhs(X, y)
    Xd = X.toarray() if hasattr(X, "toarray") else np.asarray(X, dtype=np.float64)
    A = Xd.T @ Xd + lam * np.eye(Xd.shape[1])
    return sla.cho_solve(sla.cho_factor(A, lower=True), b)


def solve_tlfcg(X, y, lam, labels, F_C, m=1, steps=2, tol=1e-10, max_iter=10_000,
                fixed_iters=None, rhs_is_b=False, jacobi=False, P=None):
    """Flexible CG (truncation m) with the two-level preconditioner whose
    pre-smoother is `steps` iterations of CG (Jacobi-preconditioned with
    `jacobi`): the configuration of the paper's experiments.  P replaces the
    adjusted square-root average prolongation when given."""
    from . import operator as op
    from . import precond
    b = np.asarray(y, dtype=np.float64) if rhs_is_b else op.rhs(X, y)
    tl = precond.TwoLevel(X, lam, labels, F_C, omega=0.0, P=P)
    return fcg(lambda v: op.apply_A(X, lam, v), b, lambda r, i: tl.rougher(r, steps, jacobi), m=m, tol=tol,
               max_iter=max_iter, fixed_iters=fixed_iters)
