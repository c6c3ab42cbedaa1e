"""Full-size parity on the 200,000 x 100,000 binary fingerprint workload
(12.0 M nonzeros, Zipf(1.1) column popularity), in the launch configuration
the benchmark times.

The oracle cannot run k-means at this size in seconds, so clustering is
checked through a property that holds at any size: after Lloyd converges,
every feature's label is the exact nearest cluster mean of the final
clusters (checked with exact integers on a sample of features, including
the most popular ones).  Solves use a seeded aggregation from datagen so the
oracle can run them too."""
import numpy as np
import pytest
import scipy.sparse as sp

import datagen
from oracle import kmeans, krylov, operator as op, precond

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rr():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1806_05826_amd as rr
    return rr


@pytest.fixture(scope="module")
def big():
    print("[fullsize] generating 200000 x 100000, 60 nnz/row", flush=True)
    return datagen.chembl_like()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_fullsize_operator_exact(rr, big):
    R = rr.Ridge(big.X)
    v = np.random.default_rng(3).integers(-40, 40, size=big.X.shape[1]).astype(np.float64)
    got = host(R.apply_operator(2.0, v))
    assert np.array_equal(got, op.apply_A(big.X, 2.0, v))
    b = host(R.apply_rhs(big.y))
    assert np.allclose(b, op.rhs(big.X, big.y), rtol=1e-13, atol=1e-11)
    R.close()


def test_fullsize_valued_operator(rr, big):
    """The same pattern with standard-normal FP64 values (the HBM-resident
    operator the benchmark times): every output against the oracle's
    operator, relative to |X|^T |X| |v| (both sides add up to tens of
    thousands of FP64 terms per output, in different orders)."""
    X = big.X.tocsr().astype(np.float64)
    X.data = np.random.default_rng(8).standard_normal(X.nnz)
    R = rr.Ridge(X, binary=False)
    v = np.random.default_rng(9).standard_normal(X.shape[1])
    got = host(R.apply_operator(0.5, v))
    ref = op.apply_A(X, 0.5, v)
    scale = abs(X).T @ (abs(X) @ np.abs(v)) + 0.5 * np.abs(v)
    err = np.max(np.abs(got - ref) / scale)
    print(f"[fullsize] valued operator: max error / |X|^T|X||v| = {err:.2e}", flush=True)
    assert err <= 1e-12
    R.close()


def test_fullsize_kmeans_fixed_point(rr, big):
    print("[fullsize] GPU k-means k=1000", flush=True)
    R = rr.Ridge(big.X, n_clusters=1000, seed=5826)
    info = R.info
    print(f"[fullsize] setup {info['setup_ms']:.0f} ms (k-means {info['kmeans_ms']:.0f} ms), "
          f"centres {info['n_centres']}, Lloyd passes {info['kmeans_iters']}, F_C {info['n_coarse']}",
          flush=True)
    assert info["kmeans_iters"] < 100, "Lloyd did not converge; fixed-point check needs convergence"
    lab = host(R.labels()).astype(np.int64)
    fc = info["n_coarse"]
    assert lab.min() == 0 and lab.max() == fc - 1
    n = np.bincount(lab, minlength=fc).astype(np.int64)
    assert np.all(n > 0)
    Xi = big.X.astype(np.int64).tocsr()
    Pu = sp.csr_matrix((np.ones(lab.size, dtype=np.int64), (np.arange(lab.size), lab)),
                       shape=(lab.size, fc))
    S = (Xi @ Pu).tocsr()
    Q = np.asarray(S.multiply(S).sum(axis=0)).ravel().astype(np.int64)
    colnnz = np.diff(big.X.tocsc().indptr)
    rng = np.random.default_rng(0)
    sample = np.unique(np.concatenate([np.argsort(-colnnz)[:20], rng.choice(lab.size, 300, replace=False)]))
    XcT = Xi.T.tocsr()[sample]
    H = np.asarray((XcT @ S).todense(), dtype=np.int64)       # h_js for the sample
    num = Q[None, :] - 2 * n[None, :] * H
    best = kmeans.exact_argmin(num, n * n, np.ones(fc, dtype=bool))
    assert np.array_equal(best, lab[sample])
    # K = P^T X^T X P on the sampled rows
    K = host(R.coarse_gram())
    sel = lab[sample[:8]]
    StS_rows = (S.tocsc()[:, sel].T @ S).toarray().astype(np.float64)
    sc = 1.0 / np.sqrt(n.astype(np.float64))
    Kref = StS_rows * sc[sel, None] * sc[None, :]
    assert np.allclose(K[sel], Kref, rtol=1e-14, atol=0)
    R.close()


@pytest.fixture(scope="module")
def solver_random_labels(rr, big):
    lab = datagen.random_labels(big.X.shape[1], 1000, 11)
    R = rr.Ridge(big.X, labels=lab)
    return R, lab


@pytest.mark.parametrize("lam", [1e-2, 1.0, 100.0])
def test_fullsize_solve(rr, big, solver_random_labels, lam):
    R, lab = solver_random_labels
    fc = 1000
    print(f"[fullsize] solve lambda={lam}", flush=True)
    w, info = R.solve(lam, big.y, precond="vcycle", tol=1e-10, max_iter=2000)
    assert info["status"] == 0 and info["relres"] <= 1e-10
    # the true residual by the oracle's operator, a property at any size
    b = op.rhs(big.X, big.y)
    wn = host(w)
    res = np.linalg.norm(b - op.apply_A(big.X, lam, wn)) / np.linalg.norm(b)
    assert res <= 2e-10
    assert abs(res - info["true_relres"]) <= 1e-12
    # iteration count inside the oracle's rounding spread (diagonal perturbed
    # by at most 2 ulp), with 2 % slack for the small ensemble
    omega = op.omega_gershgorin(big.X, lam)
    tl = precond.TwoLevel(big.X, lam, lab, fc, omega)
    A = lambda v: op.apply_A(big.X, lam, v)
    D0 = tl.D.copy()
    its = []
    rng = np.random.default_rng(1)
    Ac0 = tl.Ac.copy()
    plain = tl.coarse_correction
    for t in range(4):
        tl.D = D0
        tl.coarse_correction = plain
        if t in (1, 2):   # coarse solve through an explicit inverse
            L0 = np.linalg.cholesky(Ac0)
            Ai = np.linalg.inv(Ac0) if t == 1 else np.linalg.inv(L0).T @ np.linalg.inv(L0)
            tl.coarse_correction = lambda r, Ai=Ai: tl.P @ (Ai @ (tl.P.T @ r))
        elif t == 3:      # diagonal and A_c to within 2 ulp, A_c symmetric
            tl.D = D0 * (1.0 + (rng.random(D0.size) - 0.5) * 4 * 2**-53)
            E = (rng.random(Ac0.shape) - 0.5) * 4 * 2**-53
            tl.Ac = Ac0 * (1.0 + 0.5 * (E + E.T))
            tl.L = np.linalg.cholesky(tl.Ac)
        its.append(krylov.pcg(A, b, tl.vcycle, tol=1e-10, max_iter=2000)[1].iters)
    tl.coarse_correction = plain
    slack = 1 + int(0.02 * max(its))
    print(f"[fullsize] lambda={lam}: GPU {info['iters']} iterations, oracle ensemble {sorted(its)} "
          f"(spread {min(its)}..{max(its)}, band +-{slack})", flush=True)
    if min(its) == max(its):   # no spread: the plain +-1 rule
        assert abs(info["iters"] - its[0]) <= 1, (info["iters"], its)
    assert min(its) - slack <= info["iters"] <= max(its) + slack, (info["iters"], its)
    # oracle at equal iteration count once converged (1e-13)
    tl.D = D0
    tl.Ac = Ac0
    tl.L = np.linalg.cholesky(Ac0)
    x_t, inf_t = krylov.pcg(A, b, tl.vcycle, tol=1e-13, max_iter=2000)
    assert inf_t.status == krylov.OK
    w, info = R.solve(lam, big.y, precond="vcycle", fixed_iters=inf_t.iters)
    assert np.linalg.norm(host(w) - x_t) <= 1e-10 * np.linalg.norm(x_t)


@pytest.mark.parametrize("lam", [1e-2, 1.0, 100.0])
def test_fullsize_mixed_precision(rr, big, solver_random_labels, lam):
    """FP32 inner solves inside FP64 refinement reach the FP64 solution: the
    reference is the oracle's PCG
    (FP64, same aggregation; converged to 1e-14); the refined solution is
    asserted within 1e-10 relative error of it."""
    R, lab = solver_random_labels
    fc = 1000
    print(f"[fullsize] mixed precision lambda={lam}", flush=True)
    x_ref, inf_ref = krylov.solve(big.X, big.y, lam, "vcycle", lab, fc, tol=1e-14, max_iter=3000)
    assert inf_ref.status == krylov.OK
    w, info = R.solve(lam, big.y, precond="vcycle", precision="f32_ir", tol=1e-13, max_iter=3000)
    err = np.linalg.norm(host(w) - x_ref) / np.linalg.norm(x_ref)
    print(f"[fullsize] mixed lambda={lam}: {info['ir_steps']} steps, {info['iters']} inner "
          f"iterations, residual {info['relres']:.1e}, error {err:.1e}", flush=True)
    assert info["status"] == 0 and info["ir_steps"] >= 2
    assert err <= 1e-10


@pytest.fixture(scope="module")
def kmeans_solver(rr, big):
    R = rr.Ridge(big.X, n_clusters=1000, seed=5826)
    lab = host(R.labels()).astype(np.int64)
    return R, lab, R.info["n_coarse"]


@pytest.mark.parametrize("lam", [1.0, 100.0])
def test_fullsize_solve_on_kmeans_labels(rr, big, kmeans_solver, lam):
    """The benchmark's aggregation (GPU k-means, k = 1000): at the oracle's
    converged iteration count (relative residual 1e-13) the GPU iterate
    equals the oracle's V(1,1) PCG iterate on the same labels to 1e-10, and
    the natural-stop count at 1e-10 lies within one of the oracle's."""
    R, lab, fc = kmeans_solver
    print(f"[fullsize] k-means labels, lambda={lam}", flush=True)
    omega = op.omega_gershgorin(big.X, lam)
    tl = precond.TwoLevel(big.X, lam, lab, fc, omega)
    A = lambda v: op.apply_A(big.X, lam, v)
    b = op.rhs(big.X, big.y)
    x_t, inf_t = krylov.pcg(A, b, tl.vcycle, tol=1e-13, max_iter=2000)
    assert inf_t.status == krylov.OK
    w, info = R.solve(lam, big.y, precond="vcycle", fixed_iters=inf_t.iters)
    err = np.linalg.norm(host(w) - x_t) / np.linalg.norm(x_t)
    k10 = next(k for k, h in enumerate(inf_t.history) if h <= 1e-10)
    _, i10 = R.solve(lam, big.y, precond="vcycle", tol=1e-10, max_iter=2000)
    print(f"[fullsize] k-means lambda={lam}: {inf_t.iters} iterations to 1e-13, error {err:.1e}; "
          f"relres 1e-10 at {k10} (oracle) / {i10['iters']} (GPU)", flush=True)
    assert err <= 1e-10
    assert abs(i10["iters"] - k10) <= 1


@pytest.mark.parametrize("lam", [1e-2, 100.0])
def test_fullsize_fp32_cycle(rr, big, solver_random_labels, lam):
    """FP64 flexible CG with the V(1,1) cycle in FP32 reaches the oracle's
    FP64 solution (same aggregation, converged to 1e-14) to relative error
    1e-10, the accuracy the plain FP64 path is measured at: it stops on the
    error to that solution, which it must reach, and the error recomputed on
    the host from the returned w confirms it.  (At equal residuals the two
    cycles' iterates differ by up to kappa(A) times the residual: the FP32
    cycle's coarse correction is less exact, so more of what remains lies in
    the smallest eigenvalues' directions; a residual bar would not state the
    accuracy reached.)"""
    R, lab = solver_random_labels
    print(f"[fullsize] FP32 cycle lambda={lam}", flush=True)
    x_ref, inf_ref = krylov.solve(big.X, big.y, lam, "vcycle", lab, 1000, tol=1e-14, max_iter=3000)
    assert inf_ref.status == krylov.OK
    xr = torch.as_tensor(x_ref, dtype=torch.float64, device="cuda")
    kw = dict(precond="vcycle", krylov="fcg", fcg_m=1, tol=1e-15, max_iter=3000, x_ref=xr, err_tol=1e-10)
    w, info = R.solve(lam, big.y, precision="f32_cycle", **kw)
    w64, i64 = R.solve(lam, big.y, **kw)
    err = np.linalg.norm(host(w) - x_ref) / np.linalg.norm(x_ref)
    err64 = np.linalg.norm(host(w64) - x_ref) / np.linalg.norm(x_ref)
    print(f"[fullsize] FP32 cycle lambda={lam}: {info['iters']} iterations to error {err:.2e} "
          f"(FP64 cycle: {i64['iters']} iterations, error {err64:.2e})", flush=True)
    assert info["status"] == 0 and i64["status"] == 0
    assert err <= 1e-10 and err64 <= 1e-10


def test_fullsize_leader_follower_rule(rr, big):
    """Leader-follower clustering at the benchmark's tolerance (24): the
    oracle's dense Gram matrix does not fit at this size, so the rule is
    checked where it is defined, with exact integer distances: leaders are
    created in feature order and each is at least the tolerance away from
    every earlier leader; a follower joins the nearest earlier leader (the
    first of equal ones), strictly inside the tolerance.  Checked on the
    first 64 features, 256 drawn ones and 64 drawn leaders; then the V(1,1)
    solve on this aggregation equals the oracle's at its converged count."""
    tol = 24.0
    R = rr.Ridge(big.X, lf_tolerance=tol)
    fc = R.info["n_coarse"]
    lab = host(R.labels()).astype(np.int64)
    lead = host(R.centres())[:fc].astype(np.int64)
    print(f"[fullsize] leader-follower tol {tol}: F_C {fc}", flush=True)
    F = big.X.shape[1]
    assert np.all(np.diff(lead) > 0) and lead[0] == 0
    assert np.array_equal(lab[lead], np.arange(fc)) and lab.min() >= 0 and lab.max() < fc
    Xc = sp.csc_matrix(big.X, dtype=np.int64)
    c = np.asarray(Xc.sum(axis=0)).ravel()
    rng = np.random.default_rng(17)
    sample = np.unique(np.r_[np.arange(64), rng.choice(F, 256, replace=False), rng.choice(lead, 64)])
    G = (Xc[:, sample].T @ Xc[:, lead]).toarray()   # exact integer inner products
    for row, j in enumerate(sample):
        k = int(np.searchsorted(lead, j))            # leaders created before j: lead[:k]
        d2 = c[j] + c[lead[:k]] - 2 * G[row, :k]
        if k < fc and lead[k] == j:                  # j leads cluster k
            assert k == 0 or d2.min() >= tol * tol, (j, k)
        else:
            s = int(np.argmin(d2))
            assert lab[j] == s and d2[s] < tol * tol, (j, lab[j], s)
    lam = 1.0
    omega = op.omega_gershgorin(big.X, lam)
    tl = precond.TwoLevel(big.X, lam, lab, fc, omega)
    A = lambda v: op.apply_A(big.X, lam, v)
    x_t, inf_t = krylov.pcg(A, op.rhs(big.X, big.y), tl.vcycle, tol=1e-13, max_iter=2000)
    assert inf_t.status == krylov.OK
    w, info = R.solve(lam, big.y, precond="vcycle", fixed_iters=inf_t.iters)
    err = np.linalg.norm(host(w) - x_t) / np.linalg.norm(x_t)
    print(f"[fullsize] leader-follower solve: {inf_t.iters} iterations, error {err:.1e}", flush=True)
    assert err <= 1e-10
    R.close()


def test_fullsize_least_squares_interpolation(rr, big):
    """Least-squares interpolation on the leader-follower aggregation at the
    benchmark's tolerance, from 8 seeded prototype vectors: the weights p
    against the oracle's at every feature, the coarse Gram matrix
    P^T X^T X P against its definition (sparse products, exact for the
    pattern, FP64 for the weights), and a solve on it to relative residual
    1e-10 whose true residual the oracle's operator confirms."""
    from oracle import interp
    R = rr.Ridge(big.X, lf_tolerance=24.0, lambda_slots=2)
    fc = R.info["n_coarse"]
    lab = host(R.labels()).astype(np.int64)
    F = big.X.shape[1]
    V = np.random.default_rng(23).standard_normal((F, 8))
    beta = 1.0
    eta = interp.prototype_energies(big.X, V, beta)
    p_or = interp.ls_weights(V, eta, lab, fc, interp.representatives(lab, fc))
    p = host(R.set_interpolation(V, beta))
    err_p = np.max(np.abs(p - p_or)) / np.max(np.abs(p_or))
    print(f"[fullsize] least-squares weights: F_C {fc}, max error {err_p:.1e}", flush=True)
    assert np.allclose(p, p_or, rtol=1e-10, atol=1e-12 * np.abs(p_or).max())
    Pm = interp.ls_prolongation(lab, fc, p_or)
    Xs = sp.csr_matrix(big.X, dtype=np.float64) @ Pm
    Kref = (Xs.T @ Xs).toarray()
    K = host(R.coarse_gram()).reshape(fc, fc)
    assert np.allclose(K, Kref, rtol=1e-10, atol=1e-11 * np.abs(Kref).max())
    lam = 1.0
    w, info = R.solve(lam, big.y, precond="vcycle", tol=1e-10, max_iter=2000)
    b = op.rhs(big.X, big.y)
    wh = host(w)
    rel = np.linalg.norm(b - op.apply_A(big.X, lam, wh)) / np.linalg.norm(b)
    print(f"[fullsize] least-squares V(1,1): {info['iters']} iterations, true residual {rel:.1e}",
          flush=True)
    assert info["status"] == 0 and rel <= 2e-10
    R.close()
