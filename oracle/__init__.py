"""CPU oracle for two-level preconditioned CG on the regularized normal
equations (X^T X + lambda I) w = X^T y (the paper's eq. for the regularized
normal equations and its ridge-regression solution).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, FP64 statement
of what the GPU library computes.  Only the test suite, the smoke check and
the CPU-baseline leg of the benchmark may import it; the GPU library never
does, and it shares no code with the GPU library (no kernels, headers,
helpers or constant tables).  Inputs come from ``datagen`` (random draws
only) or from the caller.

Notation: the paper's regularization parameter beta is called ``lam`` here.
N samples, F features, F_C coarse size; A = X^T X + lam I; P is the F x F_C
prolongation with one nonzero 1/sqrt(n_s) per row (the adjusted square-root
average interpolation); A_c = P^T A P.

Modules
-------
splitmix64  the SplitMix64 generator (Steele, Lea & Flood 2014) that drives
            the k-means++ draws on both sides
operator    A v, b = X^T y, the Jacobi diagonal and the smoother weight
kmeans      k-means++ seeding and Lloyd iterations over feature columns,
            exact integer arithmetic for binary X
coarse      P, K = P^T X^T X P, A_c, its Cholesky factor
precond     z = B r for CG (none), Jacobi, the two-level V(1,1) cycle and the
            additive two-level form
krylov      PCG and flexible CG with truncation
refine      iterative refinement around a lower-precision inner solve
mlp         the learned coarse-correction network (forward, backward, loss)
leader      leader-follower clustering of the feature columns
interp      least-squares interpolation weights from prototype vectors

Every function is pinned by tests under ``tests/`` that check it against
closed forms, brute force, invariants or library routines.
"""
from .splitmix64 import SplitMix64
from . import operator, kmeans, coarse, precond, krylov

__all__ = ["SplitMix64", "operator", "kmeans", "coarse", "precond", "krylov"]
