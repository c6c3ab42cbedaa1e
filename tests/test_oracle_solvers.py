"""Pins for the oracle's preconditioners and Krylov solvers: the ridge
solution from an independent least-squares route, closed forms, the
ideal-case one-step convergence, SPD-ness, monotone A-norm error and the
flexible-CG / PCG equivalence."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import datagen
from oracle import coarse, kmeans, krylov, operator as op, precond


def _lstsq_ridge(Xd, y, lam):
    """argmin ||X w - y||^2 + lam ||w||^2 through the augmented system
    [X; sqrt(lam) I] w = [y; 0] (QR/SVD least squares, no normal
    equations)."""
    F = Xd.shape[1]
    Aug = np.vstack([Xd, np.sqrt(lam) * np.eye(F)])
    rhs = np.concatenate([y, np.zeros(F)])
    return sla.lstsq(Aug, rhs)[0]


@pytest.fixture(scope="module")
def tiny():
    P = datagen.tiny_sparse()
    lab, fc, _, _ = kmeans.kmeans_features(P.X, 50, 42)
    return P, lab, fc


@pytest.mark.parametrize("method", ["none", "jacobi", "vcycle", "additive"])
def test_solution_matches_least_squares(tiny, method):
    P, lab, fc = tiny
    lam = 1.0
    w_ls = _lstsq_ridge(P.X.toarray(), P.y, lam)
    Xd = P.X.toarray()
    kappa = np.linalg.cond(Xd.T @ Xd + lam * np.eye(Xd.shape[1]))
    w, info = krylov.solve(P.X, P.y, lam, method, lab, fc, tol=1e-10)
    assert info.status == krylov.OK
    assert info.relres <= 1e-10
    assert np.linalg.norm(w - w_ls) / np.linalg.norm(w_ls) <= kappa * 1e-10
    assert info.true_relres <= 2e-10


def test_iteration_ordering(tiny):
    """Two-level needs fewer iterations than CG (the paper's overview
    table)."""
    P, lab, fc = tiny
    its = {m: krylov.solve(P.X, P.y, 1.0, m, lab, fc, tol=1e-10)[1].iters
           for m in ["none", "jacobi", "vcycle"]}
    assert its["vcycle"] < its["jacobi"] < its["none"]


def test_disjoint_supports_closed_form():
    """X^T X diagonal: w_j = x_j^T y / (c_j + lam); Jacobi-PCG is exact in
    one step."""
    rng = np.random.default_rng(3)
    N, F = 40, 8
    Xd = np.zeros((N, F))
    rows = rng.permutation(N)
    for j in range(F):
        Xd[rows[5 * j:5 * j + 5], j] = 1.0
    y = rng.standard_normal(N)
    lam = 0.7
    w_cf = (Xd.T @ y) / ((Xd ** 2).sum(axis=0) + lam)
    w, info = krylov.solve(sp.csr_matrix(Xd), y, lam, "jacobi", tol=1e-14)
    assert info.iters == 1
    assert np.allclose(w, w_cf, rtol=1e-14, atol=0)


def test_zero_matrix_gives_zero():
    X = sp.csr_matrix((10, 6))
    w, info = krylov.solve(X, np.ones(10), 1.0, "jacobi")
    assert info.iters == 0 and np.all(w == 0)


def test_ideal_case_one_iteration():
    """Duplicated columns: range(P) holds b = X^T y and is invariant under A
    and D, so the V-cycle is exact there and PCG stops after one step."""
    X, group = datagen.duplicated_columns(40, [3, 4, 2, 5], 0.3, seed=8)
    lab, fc, _, _ = kmeans.kmeans_features(X, 4, 3)
    y = np.random.default_rng(1).standard_normal(40)
    w, info = krylov.solve(X, y, 0.5, "vcycle", lab, fc, tol=1e-12)
    assert info.iters == 1
    w_ls = _lstsq_ridge(X.toarray(), y, 0.5)
    assert np.linalg.norm(w - w_ls) <= 1e-11 * np.linalg.norm(w_ls)


def test_singleton_clusters_one_iteration():
    """labels = 0..F-1: P = I, A_c = A, the coarse correction is exact."""
    P = datagen.tiny_sparse()
    F = P.X.shape[1]
    lab = np.arange(F, dtype=np.int32)
    w, info = krylov.solve(P.X, P.y, 1.0, "vcycle", lab, F, tol=1e-12)
    assert info.iters == 1


def _dense_B(apply_B, F):
    return np.column_stack([apply_B(e) for e in np.eye(F)])


@pytest.mark.parametrize("kind", ["jacobi", "vcycle", "additive"])
def test_preconditioner_spd(kind):
    X = datagen.zipf_binary_csr(120, 40, 6, 1.1, 31)
    lam = 0.3
    lab = datagen.random_labels(40, 6, 2)
    omega = op.omega_gershgorin(X, lam)
    B, _ = precond.make(kind, X, lam, lab, 6, omega)
    M = _dense_B(B, 40)
    assert np.linalg.norm(M - M.T) <= 1e-12 * np.linalg.norm(M)
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0


def test_vcycle_error_propagation_matches_paper_form():
    """I - B A = (I - S A)(I - P A_c^-1 P^T A)(I - S A) with S = omega D^-1."""
    X = datagen.zipf_binary_csr(100, 30, 5, 1.1, 41)
    lam = 0.8
    lab = datagen.random_labels(30, 5, 4)
    omega = op.omega_gershgorin(X, lam)
    B, _ = precond.make("vcycle", X, lam, lab, 5, omega)
    Xd = X.toarray()
    A = Xd.T @ Xd + lam * np.eye(30)
    S = omega * np.diag(1.0 / np.diag(A))
    Pm = coarse.prolongation(lab, 5).toarray()
    Ac = Pm.T @ A @ Pm
    I = np.eye(30)
    T = (I - S @ A) @ (I - Pm @ np.linalg.solve(Ac, Pm.T @ A)) @ (I - S @ A)
    assert np.allclose(I - _dense_B(B, 30) @ A, T, atol=1e-12)


def test_A_is_spd():
    X = datagen.zipf_binary_csr(30, 50, 4, 1.1, 5)   # N < F: null space
    lam = 0.25
    Xd = X.toarray()
    ev = np.linalg.eigvalsh(Xd.T @ Xd + lam * np.eye(50))
    assert ev.min() >= lam * (1 - 1e-12)
    assert np.isclose(ev.min(), lam)


@pytest.mark.parametrize("kind", ["none", "jacobi", "vcycle"])
def test_monotone_A_norm_error(kind):
    X = datagen.zipf_binary_csr(200, 60, 6, 1.1, 51)
    lam = 0.1
    y = np.random.default_rng(2).standard_normal(200)
    lab = datagen.random_labels(60, 8, 5)
    Xd = X.toarray()
    A = Xd.T @ Xd + lam * np.eye(60)
    wst = np.linalg.solve(A, Xd.T @ y)
    errs = []
    for k in range(0, 25):
        w, _ = krylov.solve(X, y, lam, kind, lab, 8, fixed_iters=k)
        e = w - wst
        errs.append(np.sqrt(e @ A @ e))
    scale = np.sqrt(wst @ A @ wst)
    assert all(b <= a + 1e-14 * scale for a, b in zip(errs, errs[1:]))


def test_fcg1_reproduces_pcg():
    P = datagen.tiny_sparse()
    lam = 1.0
    lab, fc, _, _ = kmeans.kmeans_features(P.X, 50, 42)
    omega = op.omega_gershgorin(P.X, lam)
    B, _ = precond.make("vcycle", P.X, lam, lab, fc, omega)
    b = op.rhs(P.X, P.y)
    A = lambda v: op.apply_A(P.X, lam, v)
    # equal in exact arithmetic; in FP64 the rounding differences are
    # amplified mid-solve (kappa ~ 5e3) and vanish again at convergence
    for k in (1, 2, 3, 5, 8, 12, 16, 20, 24):
        xp, _ = krylov.pcg(A, b, B, fixed_iters=k)
        xf, _ = krylov.fcg(A, b, lambda r, i: B(r), m=1, fixed_iters=k)
        rel = np.linalg.norm(xp - xf) / np.linalg.norm(xp)
        assert rel <= (1e-13 if k <= 5 or k >= 20 else 1e-8)


def test_fcg_truncation_schedule():
    """m_i = max(1, i mod (m+1)) directions are kept: with m = 3 FCG stays
    exact against a variable preconditioner on a tiny SPD system."""
    rng = np.random.default_rng(4)
    M = rng.standard_normal((12, 12))
    A = M @ M.T + 12 * np.eye(12)
    b = rng.standard_normal(12)
    Bs = [np.diag(1.0 / (np.diag(A) * (1 + 0.1 * i))) for i in range(40)]
    x, info = krylov.fcg(lambda v: A @ v, b, lambda r, i: Bs[i] @ r, m=3, tol=1e-12)
    assert info.status == krylov.OK
    assert np.allclose(A @ x, b, atol=1e-10)


def test_stopping_rule_is_first_crossing(tiny):
    P, lab, fc = tiny
    w, info = krylov.solve(P.X, P.y, 1.0, "vcycle", lab, fc, tol=1e-8)
    assert info.history[-1] <= 1e-8 < info.history[-2]


def test_not_converged_and_breakdown():
    P = datagen.tiny_sparse()
    w, info = krylov.solve(P.X, P.y, 1.0, "none", tol=1e-10, max_iter=5)
    assert info.status == krylov.NOT_CONVERGED and info.iters == 5
    lab = datagen.random_labels(500, 50, 1)
    # omega far above 2 / rho(D^-1 A): the V-cycle is indefinite
    w, info = krylov.solve(P.X, P.y, 1.0, "vcycle", lab, 50, omega=50.0, tol=1e-10)
    assert info.status == krylov.BREAKDOWN


# --- the cluster-aligned block smoother ----------------------------------------

def test_block_smoother_structure_and_point_limit():
    """Blocks never cross a cluster, cover every feature once in increasing
    order, hold <= 32 features; with blocks of one feature the block
    smoother is the point Jacobi smoother."""
    import datagen
    from oracle import precond, operator as op
    P = datagen.tiny_sparse()
    F = P.X.shape[1]
    lab = datagen.random_labels(F, 7, 3)
    blocks = precond.smoother_blocks(lab, 7)
    allf = np.concatenate(blocks)
    assert np.array_equal(np.sort(allf), np.arange(F))
    assert all(b.size <= 32 and np.all(np.diff(b) > 0) and np.unique(lab[b]).size == 1 for b in blocks)
    ones = precond.smoother_blocks(lab, 7, size=1)
    inv = precond.block_inverses(P.X, 0.5, ones)
    r = np.random.default_rng(2).standard_normal(F)
    assert np.allclose(precond.block_apply(ones, inv, r), r / op.jacobi_diagonal(P.X, 0.5),
                       rtol=1e-14, atol=0)


def test_block_smoother_exact_on_one_block():
    """F <= 32 in one cluster: D_B = A, so with omega = 1 the pre-smoothing
    already solves A e = r and V(1,1) PCG ends after one iteration."""
    import datagen
    from oracle import krylov
    X = datagen.zipf_binary_csr(80, 24, 5, 1.1, 6)
    y = np.random.default_rng(7).standard_normal(80)
    lab = np.zeros(24, dtype=np.int64)
    x, inf = krylov.solve(X, y, 0.3, "vcycle", lab, 1, omega=1.0, tol=1e-12, smoother="block")
    assert inf.iters == 1
    ref = krylov.reference_solution(X, y, 0.3)
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)


def test_block_smoother_spd_and_weight():
    """The block V(1,1) preconditioner is SPD on a tiny problem with the
    power weight, and the weight's estimate is within 2 % of rho(D_B^-1 A)
    from the eigenvalues."""
    import datagen
    from oracle import precond, operator as op
    P = datagen.tiny_sparse()
    F = P.X.shape[1]
    lab = datagen.random_labels(F, 9, 4)
    lam = 0.7
    blocks = precond.smoother_blocks(lab, 9)
    inv = precond.block_inverses(P.X, lam, blocks)
    om = precond.block_omega(P.X, lam, blocks, inv, 0x5eed)
    A = P.X.T @ P.X
    A = np.asarray(A.todense()) + lam * np.eye(F)
    DBinv = np.zeros((F, F))
    for B, Gi in zip(blocks, inv):
        DBinv[np.ix_(B, B)] = Gi
    rho = np.max(np.abs(np.linalg.eigvals(DBinv @ A)))
    assert abs(1.0 / (1.1 * om) - rho) <= 0.02 * rho
    tl = precond.TwoLevel(P.X, lam, lab, 9, om, "block")
    Bm = np.stack([tl.vcycle(e) for e in np.eye(F)], axis=1)
    assert np.abs(Bm - Bm.T).max() <= 1e-12 * np.abs(Bm).max()
    assert np.linalg.eigvalsh(0.5 * (Bm + Bm.T)).min() > 0


# --- the CG rougher of the paper's experiments (TLFCG) -----------------------------

def test_cg_rougher_is_the_krylov_optimum():
    """Two CG steps from 0 give the A-orthogonal (Galerkin) projection of the
    solution onto span{r, A r}, and the returned residual is r - A e."""
    from oracle import precond
    rng = np.random.default_rng(11)
    M = rng.standard_normal((30, 30))
    A = M @ M.T + 0.5 * np.eye(30)
    r = rng.standard_normal(30)
    e, res = precond.cg_rougher(lambda v: A @ v, r, 2)
    V = np.stack([r, A @ r], axis=1)
    c = np.linalg.solve(V.T @ A @ V, V.T @ r)
    assert np.allclose(e, V @ c, rtol=1e-10, atol=1e-12)
    assert np.allclose(res, r - A @ e, rtol=1e-10, atol=1e-12)


def test_cg_rougher_exact_on_two_eigenvalues():
    """A with two distinct eigenvalues: two CG steps solve A e = r exactly,
    so the coarse correction of the residual adds nothing."""
    from oracle import precond
    rng = np.random.default_rng(12)
    Q, _ = np.linalg.qr(rng.standard_normal((20, 20)))
    A = Q @ np.diag([2.0] * 9 + [7.0] * 11) @ Q.T
    r = rng.standard_normal(20)
    e, res = precond.cg_rougher(lambda v: A @ v, r, 2)
    assert np.allclose(e, np.linalg.solve(A, r), rtol=1e-12, atol=1e-12)
    assert np.linalg.norm(res) <= 1e-12 * np.linalg.norm(r)


def test_tlfcg_converges_to_the_solution():
    """TLFCG reaches the dense Cholesky solution and needs fewer iterations
    than unpreconditioned CG on a clustered tiny problem."""
    import datagen
    from oracle import kmeans, krylov
    P = datagen.tiny_sparse()
    lab, fc, _, _ = kmeans.kmeans_features(P.X, 50, 1)
    x, inf = krylov.solve_tlfcg(P.X, P.y, 1.0, lab, fc, tol=1e-12)
    ref = krylov.reference_solution(P.X, P.y, 1.0)
    assert inf.status == 0
    assert np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref)
    _, inf_cg = krylov.solve(P.X, P.y, 1.0, "none", tol=1e-12)
    assert inf.iters < inf_cg.iters


def test_jacobi_cg_rougher_is_the_preconditioned_optimum():
    """Jacobi-PCG steps give the A-orthogonal projection onto the
    preconditioned Krylov space span{D^-1 r, D^-1 A D^-1 r}."""
    from oracle import precond
    rng = np.random.default_rng(13)
    M = rng.standard_normal((25, 25))
    A = M @ M.T + 0.5 * np.eye(25)
    D = np.diag(A).copy()
    r = rng.standard_normal(25)
    e, res = precond.cg_rougher(lambda v: A @ v, r, 2, D)
    z0 = r / D
    V = np.stack([z0, (A @ z0) / D], axis=1)
    c = np.linalg.solve(V.T @ A @ V, V.T @ r)
    assert np.allclose(e, V @ c, rtol=1e-10, atol=1e-12)
    assert np.allclose(res, r - A @ e, rtol=1e-10, atol=1e-12)


# --- the two-level forms against dense matrices built entry by entry ----------------

def _dense_prolongation(labels, F_C):
    """P[j, labels[j]] = 1 / sqrt(n_s), written one entry at a time."""
    n = [0] * F_C
    for s in labels:
        n[int(s)] += 1
    P = np.zeros((len(labels), F_C))
    for j, s in enumerate(labels):
        P[j, int(s)] = 1.0 / np.sqrt(n[int(s)])
    return P


def _dense_A(X, lam):
    Xd = X.toarray()
    return Xd.T @ Xd + lam * np.eye(Xd.shape[1])


def test_additive_is_weighted_jacobi_plus_galerkin_correction():
    """B = omega D^-1 + P (P^T A P)^-1 P^T, every matrix formed densely."""
    X = datagen.zipf_binary_csr(120, 40, 6, 1.1, 31)
    lam = 0.3
    lab = datagen.random_labels(40, 6, 2)
    omega = op.omega_gershgorin(X, lam)
    A = _dense_A(X, lam)
    P = _dense_prolongation(lab, 6)
    ref = omega * np.diag(1.0 / np.diag(A)) + P @ np.linalg.inv(P.T @ A @ P) @ P.T
    B, _ = precond.make("additive", X, lam, lab, 6, omega)
    M = _dense_B(B, 40)
    assert np.abs(M - ref).max() <= 1e-12 * np.abs(ref).max()


def test_additive_with_singleton_clusters_closed_form():
    """P = I: B = omega D^-1 + A^-1."""
    X = datagen.zipf_binary_csr(90, 25, 5, 1.1, 32)
    lam = 0.6
    lab = np.arange(25, dtype=np.int32)
    omega = 0.37
    A = _dense_A(X, lam)
    ref = omega * np.diag(1.0 / np.diag(A)) + np.linalg.inv(A)
    B, _ = precond.make("additive", X, lam, lab, 25, omega)
    M = _dense_B(B, 25)
    assert np.abs(M - ref).max() <= 1e-12 * np.abs(ref).max()


def test_rougher_with_singleton_clusters_is_the_exact_inverse():
    """P = I makes the coarse correction exact on the rougher's residual:
    z = e1 + A^-1 (r - A e1) = A^-1 r, and TLFCG stops after one iteration.
    Correcting r instead of the residual would give e1 + A^-1 r."""
    X = datagen.zipf_binary_csr(200, 60, 8, 1.1, 5)
    lam = 0.5
    lab = np.arange(60, dtype=np.int32)
    A = _dense_A(X, lam)
    tl = precond.TwoLevel(X, lam, lab, 60, op.omega_gershgorin(X, lam))
    r = np.random.default_rng(4).standard_normal(60)
    ref = np.linalg.solve(A, r)
    for steps in (1, 2, 3):
        z = tl.rougher(r, steps)
        assert np.linalg.norm(z - ref) <= 1e-11 * np.linalg.norm(ref)
    y = np.random.default_rng(5).standard_normal(200)
    _, inf = krylov.solve_tlfcg(X, y, lam, lab, 60, tol=1e-12)
    assert inf.status == krylov.OK and inf.iters == 1


def test_rougher_exact_smoothing_leaves_nothing_to_correct():
    """A with two distinct eigenvalues (orthogonal 0/1 columns of 4 and 9
    entries): two CG steps solve A e = r, the residual is zero, so z = A^-1 r
    for any aggregation; a coarse correction of r itself would add
    P A_c^-1 P^T r."""
    N, F = 80, 12
    Xd = np.zeros((N, F))
    row = 0
    for j in range(F):
        m = 4 if j % 3 else 9
        Xd[row:row + m, j] = 1.0
        row += m
    X = sp.csr_matrix(Xd)
    lam = 0.25
    lab = np.array([0, 1, 2, 0, 1, 2, 0, 1, 2, 0, 1, 2], dtype=np.int32)
    tl = precond.TwoLevel(X, lam, lab, 3, 0.5)
    r = np.random.default_rng(6).standard_normal(F)
    z = tl.rougher(r, 2)
    assert np.allclose(z, r / (Xd.sum(axis=0) + lam), rtol=1e-12, atol=0)


def test_rougher_general_case_against_dense_projection():
    """e1 = the A-orthogonal projection of A^-1 r onto span{r, A r} (two CG
    steps), then z = e1 + P (P^T A P)^-1 P^T (r - A e1), all dense."""
    X = datagen.zipf_binary_csr(150, 45, 6, 1.1, 7)
    lam = 0.4
    lab = datagen.random_labels(45, 7, 8)
    A = _dense_A(X, lam)
    P = _dense_prolongation(lab, 7)
    r = np.random.default_rng(9).standard_normal(45)
    V = np.stack([r, A @ r], axis=1)
    e1 = V @ np.linalg.solve(V.T @ A @ V, V.T @ r)
    ref = e1 + P @ np.linalg.solve(P.T @ A @ P, P.T @ (r - A @ e1))
    tl = precond.TwoLevel(X, lam, lab, 7, op.omega_gershgorin(X, lam))
    z = tl.rougher(r, 2)
    assert np.linalg.norm(z - ref) <= 1e-10 * np.linalg.norm(ref)
