"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random inputs: sparse binary feature matrices with a
Zipf column-popularity law (the shape of the binary fingerprint data set in
the paper's data table), dense block-correlated Gaussian features, targets
y = X w* + noise, batches of uneven independent problems, and a plain random
labelling of features.  It holds none of the solver's arithmetic, so the
CPU oracle and the GPU library can both be fed from it without sharing any
method code.

Every generator is a pure function of its arguments and a seed
(``numpy.random.Generator(PCG64(seed))``).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

# Seed convention: seed = BASE_SEED + 1000 * config_number.
BASE_SEED = 5826


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class SparseProblem:
    """A sparse ridge problem: X (CSR, float64 values all 1 for binary data),
    the generating weights w_true and targets y."""

    X: sp.csr_matrix
    w_true: np.ndarray
    y: np.ndarray
    binary: bool = True


def zipf_binary_csr(n_rows: int, n_cols: int, nnz_per_row: int, exponent: float,
                    seed: int, scatter_columns: bool = True) -> sp.csr_matrix:
    """Binary CSR matrix whose rows each hold exactly ``nnz_per_row`` distinct
    columns drawn with probability proportional to (rank+1)^-exponent.

    Draws are made by inverse-CDF sampling; repeated columns inside a row are
    rejected until the row holds ``nnz_per_row`` distinct columns.  With
    ``scatter_columns`` the popularity rank is mapped to a column index by a
    seeded random permutation, so popular features are spread over the index
    range rather than packed at the front.  Column indices are sorted within
    each row.  Values are 1.0 (float64).
    """
    if nnz_per_row > n_cols:
        raise ValueError("nnz_per_row > n_cols")
    rng = _rng(seed)
    weights = (np.arange(1, n_cols + 1, dtype=np.float64)) ** (-exponent)
    cdf = np.cumsum(weights)
    cdf /= cdf[-1]
    m = nnz_per_row
    out = np.empty((n_rows, m), dtype=np.int64)
    todo = np.arange(n_rows)
    n_cand = max(4 * m, 64)
    while todo.size:
        u = rng.random((todo.size, n_cand))
        cand = np.searchsorted(cdf, u, side="right")
        cand = np.minimum(cand, n_cols - 1)
        # first occurrence of each value in each row, in draw order
        order = np.argsort(cand, axis=1, kind="stable")
        sorted_vals = np.take_along_axis(cand, order, axis=1)
        first_sorted = np.ones_like(sorted_vals, dtype=bool)
        first_sorted[:, 1:] = sorted_vals[:, 1:] != sorted_vals[:, :-1]
        first = np.zeros_like(first_sorted)
        np.put_along_axis(first, order, first_sorted, axis=1)
        rank = np.cumsum(first, axis=1)          # 1-based rank among distinct
        keep = first & (rank <= m)
        ok = keep.sum(axis=1) == m
        rows_ok = todo[ok]
        vals = cand[ok][keep[ok]].reshape(-1, m)
        out[rows_ok] = vals
        todo = todo[~ok]
        n_cand *= 2
    if scatter_columns:
        perm = rng.permutation(n_cols)
        out = perm[out]
    out.sort(axis=1)
    indptr = np.arange(0, (n_rows + 1) * m, m, dtype=np.int64)
    data = np.ones(n_rows * m, dtype=np.float64)
    X = sp.csr_matrix((data, out.reshape(-1), indptr), shape=(n_rows, n_cols))
    X.has_sorted_indices = True
    return X


def targets(X, seed: int, noise_sigma: float = 0.1, n_rhs: int = 1):
    """w* ~ N(0, 1) per feature; y = X w* + N(0, noise_sigma^2) per sample."""
    rng = _rng(seed + 7)
    n, f = X.shape
    shape = (f,) if n_rhs == 1 else (f, n_rhs)
    w = rng.standard_normal(shape)
    y = np.asarray(X @ w, dtype=np.float64)
    y = y + noise_sigma * rng.standard_normal(y.shape)
    return w, y


def sparse_problem(n_rows: int, n_cols: int, nnz_per_row: int, seed: int,
                   exponent: float = 1.1, noise_sigma: float = 0.1) -> SparseProblem:
    X = zipf_binary_csr(n_rows, n_cols, nnz_per_row, exponent, seed)
    w, y = targets(X, seed, noise_sigma)
    return SparseProblem(X=X, w_true=w, y=y, binary=True)


# --- named workloads -------------------------------------------------------

def tiny_sparse(seed: int = BASE_SEED + 1000) -> SparseProblem:
    """2000 samples x 500 features, 10 distinct columns per row (2 % density),
    Zipf(1.1) popularity."""
    return sparse_problem(2000, 500, 10, seed)


def chembl_like(seed: int = BASE_SEED + 2000) -> SparseProblem:
    """200,000 samples x 100,000 binary features, 60 distinct columns per row
    (12.0 M nonzeros), Zipf(1.1) popularity: the shape of the binary
    fingerprint data set in the paper's data table."""
    return sparse_problem(200_000, 100_000, 60, seed)


def mid_sparse(seed: int = BASE_SEED + 9000, n_rows: int = 20_000,
               n_cols: int = 6_000, nnz_per_row: int = 30) -> SparseProblem:
    """A mid-size problem the CPU oracle finishes in seconds, still many
    kernel tiles wide, with ragged tails."""
    return sparse_problem(n_rows, n_cols, nnz_per_row, seed)


def block_correlated_dense(n_rows: int, n_groups: int, group_size: int,
                           rho: float, seed: int, dtype=np.float32) -> np.ndarray:
    """Dense Gaussian features with block covariance: column j of group g is
    sqrt(rho) z_g + sqrt(1-rho) eps_j, so every column has unit variance and
    correlation rho inside its group."""
    rng = _rng(seed)
    z = rng.standard_normal((n_rows, n_groups), dtype=np.float32)
    eps = rng.standard_normal((n_rows, n_groups * group_size), dtype=np.float32)
    X = np.sqrt(1.0 - rho, dtype=np.float32) * eps
    X += np.sqrt(rho, dtype=np.float32) * np.repeat(z, group_size, axis=1)
    return X.astype(dtype, copy=False)


def random_labels(n_features: int, n_clusters: int, seed: int) -> np.ndarray:
    """A seeded uniform random assignment of features to clusters (every
    cluster non-empty when n_features >= n_clusters).  Used where a solve
    needs a valid aggregation that does not depend on any clustering code."""
    rng = _rng(seed + 13)
    lab = rng.integers(0, n_clusters, size=n_features)
    if n_features >= n_clusters:
        lab[rng.permutation(n_features)[:n_clusters]] = np.arange(n_clusters)
    return lab.astype(np.int32)


def duplicated_columns(n_rows: int, group_sizes, density: float, seed: int,
                       distinct_norms: bool = False) -> tuple[sp.csr_matrix, np.ndarray]:
    """An 'ideal' data set: group g holds group_sizes[g] identical copies of
    one random binary column.  Returns (X, group_of_column).  Columns are
    shuffled so groups are not contiguous."""
    rng = _rng(seed)
    cols = []
    group = []
    for g, n in enumerate(group_sizes):
        while True:
            v = (rng.random(n_rows) < density).astype(np.float64)
            if v.sum() > 0:
                break
        if distinct_norms:
            # make column norms differ between groups: add g extra ones
            zeros = np.flatnonzero(v == 0)
            v[zeros[:g]] = 1.0
        for _ in range(n):
            cols.append(v)
            group.append(g)
    D = np.stack(cols, axis=1)
    perm = rng.permutation(D.shape[1])
    D = D[:, perm]
    group = np.asarray(group)[perm]
    return sp.csr_matrix(D), group.astype(np.int32)


def lambdas_loguniform(n: int, lo: float, hi: float, seed: int) -> np.ndarray:
    rng = _rng(seed + 17)
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=n))


def _one_batched(args):
    n, d, m, sub, exponent = args
    P = sparse_problem(n, d, m, sub, exponent)
    return P.X.indptr, P.X.indices, P.w_true, P.y


def batched_problems(n_problems: int, seed: int, n_range=(500, 20_000),
                     d_range=(200, 8_000), density_range=(0.01, 0.05),
                     lam_range=(1e-3, 10.0), exponent: float = 1.1, workers: int = 1):
    """Independent sparse binary ridge problems of uneven size: n and d
    uniform in their ranges, density uniform, Zipf column popularity,
    lambda log-uniform.  Returns a list of (SparseProblem, lambda).  With
    ``workers`` > 1 the problems are drawn by a process pool; every problem
    has a seed of its own, so the result does not depend on ``workers``."""
    rng = _rng(seed)
    params, lams = [], []
    for p in range(n_problems):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        d = int(rng.integers(d_range[0], d_range[1] + 1))
        rho = float(rng.uniform(*density_range))
        m = max(1, int(round(rho * d)))
        lams.append(float(np.exp(rng.uniform(np.log(lam_range[0]), np.log(lam_range[1])))))
        params.append((n, d, m, seed * 1000 + p, exponent))
    if workers > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            parts = pool.map(_one_batched, params, chunksize=1)
    else:
        parts = [_one_batched(a) for a in params]
    out = []
    for (n, d, _, _, _), (indptr, indices, w, y), lam in zip(params, parts, lams):
        X = sp.csr_matrix((np.ones(indices.size), indices, indptr), shape=(n, d))
        X.has_sorted_indices = True
        out.append((SparseProblem(X=X, w_true=w, y=y, binary=True), lam))
    return out
