"""GPU parity: the HIP path, called through the C ABI, against the CPU oracle
on the same seeded inputs (datagen).  Sizes span many kernel tiles with
ragged tails; the full-size binary-fingerprint case is in
test_gpu_fullsize.py.

Bars: integer/index work bit-exact (operator on integer vectors, k-means
centres and labels); FP64 results within 1e-10 relative of the oracle at
equal iteration counts, natural-stop iteration counts within +-1."""
import numpy as np
import pytest

import datagen
from oracle import coarse, kmeans, krylov, operator as op, precond

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rr():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1806_05826_amd as rr
    return rr


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


CASES = {
    "tiny": lambda: datagen.tiny_sparse(),
    "mid": lambda: datagen.mid_sparse(),
    "ragged": lambda: datagen.sparse_problem(3001, 1237, 7, seed=77),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request, rr):
    P = CASES[request.param]()
    print(f"[case {request.param}] N={P.X.shape[0]} F={P.X.shape[1]} nnz={P.X.nnz}", flush=True)
    return request.param, P


# --- operator ------------------------------------------------------------------

def test_operator_exact_on_integers(rr, case):
    name, P = case
    R = rr.Ridge(P.X)
    v = np.random.default_rng(1).integers(-60, 60, size=P.X.shape[1]).astype(np.float64)
    got = host(R.apply_operator(3.0, v))
    ref = op.apply_A(P.X, 3.0, v)
    assert np.array_equal(got, ref)
    R.close()


def test_operator_random(rr, case):
    name, P = case
    R = rr.Ridge(P.X)
    v = np.random.default_rng(2).standard_normal(P.X.shape[1])
    got = host(R.apply_operator(0.37, v))
    ref = op.apply_A(P.X, 0.37, v)
    Xa = abs(P.X)
    scale = Xa.T @ (Xa @ np.abs(v)) + 0.37 * np.abs(v)
    assert np.all(np.abs(got - ref) <= 1e-13 * scale + 1e-300)
    b = host(R.apply_rhs(P.y))
    assert np.allclose(b, op.rhs(P.X, P.y), rtol=1e-13, atol=1e-12)
    R.close()


# --- k-means ---------------------------------------------------------------------

KM = {"tiny": (50, 42), "mid": (300, 7), "ragged": (97, 3)}


@pytest.fixture(scope="module")
def clustered(rr, case):
    name, P = case
    k, seed = KM[name]
    lab, fc, it, centres = kmeans.kmeans_features(P.X, k, seed)
    R = rr.Ridge(P.X, n_clusters=k, seed=seed)
    return name, P, R, (lab, fc, it, centres)


def test_kmeans_bit_exact(rr, clustered):
    name, P, R, (lab, fc, it, centres) = clustered
    info = R.info
    assert info["n_centres"] == len(centres)
    assert np.array_equal(host(R.centres()), centres)
    assert info["kmeans_iters"] == it
    assert info["n_coarse"] == fc
    assert np.array_equal(host(R.labels()), lab)


def test_coarse_gram_and_factor(rr, clustered):
    name, P, R, (lab, fc, it, centres) = clustered
    K = host(R.coarse_gram())
    Kref = coarse.coarse_gram(P.X, lab, fc)
    assert np.max(np.abs(K - Kref)) <= 1e-13 * np.max(np.abs(Kref))
    lam = 0.5
    L, Ai = (host(t) for t in R.coarse_factor(lam))
    Lref = coarse.cholesky(Kref + lam * np.eye(fc))
    assert np.max(np.abs(L - Lref)) <= 1e-12 * np.max(np.abs(Lref))
    Airef = np.linalg.inv(Kref + lam * np.eye(fc))
    assert np.max(np.abs(Ai - Airef)) <= 1e-10 * np.max(np.abs(Airef))


@pytest.mark.parametrize("kind", ["jacobi", "vcycle", "additive"])
def test_precond_parity(rr, clustered, kind):
    name, P, R, (lab, fc, it, centres) = clustered
    lam = 1.0
    r = np.random.default_rng(5).standard_normal(P.X.shape[1])
    omega = op.omega_gershgorin(P.X, lam)
    assert abs(R.smoother_weight(lam) - omega) <= 1e-15 * omega
    B, _ = precond.make(kind, P.X, lam, lab, fc, omega)
    z = host(R.apply_precond(lam, r, kind))
    zr = B(r)
    # K is exact on one side and FP64 products on the other: its entries
    # agree to rounding, which the coarse solve amplifies by kappa(A_c)
    kappa_c = np.linalg.cond(coarse.coarse_matrix(P.X, lab, fc, lam))
    assert np.linalg.norm(z - zr) <= 32 * kappa_c * 2**-52 * np.linalg.norm(zr)


def spread_slack(lo, hi):
    """The band around the oracle ensemble's iteration counts: +-1 where the
    ensemble agrees, else 1 + 2 % (a finite ensemble under-samples the tails
    of a nonzero spread)."""
    return 1 if lo == hi else 1 + int(0.02 * hi)


def oracle_iteration_spread(P, lam, kind, lab, fc, tol, max_iter, n=6, seed=0, fcg_m=None):
    """Iteration counts of the oracle itself under rounding-level changes:
    the coarse solve done through an explicit inverse, and the
    preconditioner's diagonal (or, for CG, an identity scaling) and the
    coarse matrix perturbed entrywise by at most 2 ulp.  FP64 Krylov
    iteration counts are only defined up to this spread (near a residual
    plateau it spans several iterations)."""
    b = op.rhs(P.X, P.y)
    A = lambda v: op.apply_A(P.X, lam, v)
    F = P.X.shape[1]
    rng = np.random.default_rng(seed)
    its = []
    omega = op.omega_gershgorin(P.X, lam) if kind in ("vcycle", "additive") else None
    for t in range(n):
        pert = np.ones(F) if t == 0 else 1.0 + (rng.random(F) - 0.5) * 4 * 2**-53
        if kind == "none":
            B = lambda r, pert=pert: r * pert
        elif kind == "jacobi":
            D = op.jacobi_diagonal(P.X, lam) * pert
            B = lambda r, D=D: r / D
        else:
            tl = precond.TwoLevel(P.X, lam, lab, fc, omega)
            if t in (1, 2):
                # the coarse solve through an explicit inverse (LU-based, or
                # from the Cholesky factor): the same solve in another
                # rounding order
                Ai = np.linalg.inv(tl.Ac) if t == 1 else np.linalg.inv(tl.L).T @ np.linalg.inv(tl.L)
                tl.coarse_correction = lambda r, tl=tl, Ai=Ai: tl.P @ (Ai @ (tl.P.T @ r))
            elif t > 2:
                # diagonal and A_c to within 2 ulp (A_c kept symmetric)
                tl.D = tl.D * pert
                E = (rng.random(tl.Ac.shape) - 0.5) * 4 * 2**-53
                tl.Ac = tl.Ac * (1.0 + 0.5 * (E + E.T))
                tl.L = coarse.cholesky(tl.Ac)
            B = tl.vcycle if kind == "vcycle" else tl.additive
        if fcg_m is None:
            _, inf = krylov.pcg(A, b, B, tol=tol, max_iter=max_iter)
        else:
            _, inf = krylov.fcg(A, b, lambda r, i, B=B: B(r), m=fcg_m, tol=tol, max_iter=max_iter)
        its.append(inf.iters)
    return min(its), max(its)


@pytest.mark.parametrize("kind", ["none", "jacobi", "vcycle", "additive"])
def test_solve_parity(rr, clustered, kind):
    name, P, R, (lab, fc, it, centres) = clustered
    lam = 1.0
    # natural stop at 1e-10: iteration count inside the oracle's rounding
    # spread, +-1; recursive and true residuals at the tolerance
    lo, hi = oracle_iteration_spread(P, lam, kind, lab, fc, 1e-10, 5000, n=8)
    w, info = R.solve(lam, P.y, precond=kind, tol=1e-10, max_iter=5000)
    assert info["status"] == 0
    slack = spread_slack(lo, hi)
    print(f"[parity {name} {kind}] {info['iters']} iterations, oracle spread {lo}..{hi}, band +-{slack}",
          flush=True)
    assert lo - slack <= info["iters"] <= hi + slack, (info["iters"], lo, hi)
    assert info["relres"] <= 1e-10
    assert info["true_relres"] <= 2e-10
    # equal iteration counts once converged (relative residual 1e-13):
    # the iterates agree to 1e-10
    x_t, inf_t = krylov.solve(P.X, P.y, lam, kind, lab, fc, tol=1e-13, max_iter=5000)
    assert inf_t.status == krylov.OK
    w, info = R.solve(lam, P.y, precond=kind, fixed_iters=inf_t.iters)
    assert info["iters"] == inf_t.iters
    assert np.linalg.norm(host(w) - x_t) <= 1e-10 * np.linalg.norm(x_t)
    # and the first step, before CG's transient amplification of rounding
    x_1, _ = krylov.solve(P.X, P.y, lam, kind, lab, fc, fixed_iters=1)
    w, info = R.solve(lam, P.y, precond=kind, fixed_iters=1)
    assert np.linalg.norm(host(w) - x_1) <= 1e-10 * np.linalg.norm(x_1)


def oracle_fcg(P, lam, kind, lab, fc, m, **kw):
    b = op.rhs(P.X, P.y)
    omega = op.omega_gershgorin(P.X, lam) if kind in ("vcycle", "additive") else None
    B, _ = precond.make(kind, P.X, lam, lab, fc, omega)
    return krylov.fcg(lambda v: op.apply_A(P.X, lam, v), b, lambda r, i: B(r), m=m, **kw)


@pytest.mark.parametrize("kind", ["none", "jacobi", "vcycle", "additive"])
@pytest.mark.parametrize("m", [1, 3])
def test_fcg_parity(rr, clustered, kind, m):
    """Flexible CG with truncation m against the oracle's flexible CG with the
    same preconditioner: converged iterates at equal counts to 1e-10, the
    first step to 1e-10, natural-stop counts inside the oracle's rounding
    spread."""
    name, P, R, (lab, fc, it, centres) = clustered
    lam = 1.0
    x_t, inf_t = oracle_fcg(P, lam, kind, lab, fc, m, tol=1e-13, max_iter=5000)
    assert inf_t.status == krylov.OK
    w, info = R.solve(lam, P.y, precond=kind, krylov="fcg", fcg_m=m, fixed_iters=inf_t.iters)
    assert info["iters"] == inf_t.iters
    assert np.linalg.norm(host(w) - x_t) <= 1e-10 * np.linalg.norm(x_t)
    x_1, _ = oracle_fcg(P, lam, kind, lab, fc, m, fixed_iters=1)
    w, info = R.solve(lam, P.y, precond=kind, krylov="fcg", fcg_m=m, fixed_iters=1)
    assert np.linalg.norm(host(w) - x_1) <= 1e-10 * np.linalg.norm(x_1)
    lo, hi = oracle_iteration_spread(P, lam, kind, lab, fc, 1e-10, 5000, n=6, fcg_m=m)
    w, info = R.solve(lam, P.y, precond=kind, krylov="fcg", fcg_m=m, tol=1e-10, max_iter=5000)
    assert info["status"] == 0
    slack = spread_slack(lo, hi)
    print(f"[parity fcg{m} {kind}] {info['iters']} iterations, oracle spread {lo}..{hi}, band +-{slack}",
          flush=True)
    assert lo - slack <= info["iters"] <= hi + slack, (info["iters"], lo, hi)
    assert info["true_relres"] <= 2e-10


def test_fcg_options(rr, clustered):
    name, P, R, _ = clustered
    with pytest.raises(rr.RRError):
        R.solve(1.0, P.y, krylov="fcg", fcg_m=17)
    with pytest.raises(rr.RRError):
        R.solve(1.0, P.y, krylov=7)
    # the ring grows on demand and a smaller m afterwards still works
    w1, i1 = R.solve(1.0, P.y, precond="vcycle", krylov="fcg", fcg_m=16, fixed_iters=20)
    w2, i2 = R.solve(1.0, P.y, precond="vcycle", krylov="fcg", fcg_m=2, fixed_iters=20)
    assert i1["iters"] == i2["iters"] == 20
    assert np.all(np.isfinite(host(w1))) and np.all(np.isfinite(host(w2)))


def test_residual_history_and_error_target(rr, clustered):
    name, P, R, (lab, fc, it, centres) = clustered
    lam = 1.0
    wst = krylov.reference_solution(P.X, P.y, lam) if P.X.shape[1] <= 4000 else None
    if wst is None:
        pytest.skip("dense reference too large")
    x, inf = krylov.solve(P.X, P.y, lam, "vcycle", lab, fc, tol=1e-13, x_ref=wst)
    hist = torch.zeros(200, dtype=torch.float64, device="cuda")
    w, info = R.solve(lam, P.y, precond="vcycle", tol=1e-10, residual_history=hist)
    h = host(hist)[: info["iters"] + 1]
    assert h[0] == 1.0 and np.all(np.isfinite(h))
    assert np.allclose(h[:3], inf.history[:3], rtol=1e-9, atol=0)
    assert abs(h[-1] - info["relres"]) <= 1e-15 and h[-1] <= 1e-10 < h[-2]
    # stop on the error against w* instead of the residual
    first = next(i for i, e in enumerate(inf.err_history) if e <= 1e-10)
    w, info = R.solve(lam, P.y, precond="vcycle", tol=1e-300, x_ref=dev(wst), err_tol=1e-10)
    assert abs(info["iters"] - first) <= 2
    assert info["err"] <= 1e-10
    assert np.linalg.norm(host(w) - wst) <= 1e-10 * np.linalg.norm(wst)


def test_deterministic(rr, clustered):
    name, P, R, _ = clustered
    w1, i1 = R.solve(1.0, P.y, precond="vcycle", fixed_iters=15)
    w2, i2 = R.solve(1.0, P.y, precond="vcycle", fixed_iters=15)
    assert torch.equal(w1, w2)


# --- aggregation given from outside ----------------------------------------------

def test_labels_in_matches_oracle(rr):
    P = datagen.mid_sparse()
    F = P.X.shape[1]
    lab = datagen.random_labels(F, 250, 9)
    lab[lab == 17] = 3            # leave cluster 17 empty: it must be dropped
    R = rr.Ridge(P.X, labels=lab)
    labc, fc = kmeans.compact(lab)
    assert R.info["n_coarse"] == fc == 249
    assert np.array_equal(host(R.labels()), labc)
    x_t, inf = krylov.solve(P.X, P.y, 0.1, "vcycle", labc, fc, tol=1e-13)
    w, info = R.solve(0.1, P.y, precond="vcycle", fixed_iters=inf.iters)
    assert np.linalg.norm(host(w) - x_t) <= 1e-10 * np.linalg.norm(x_t)


@pytest.mark.parametrize("kind", ["vcycle", "additive"])
def test_large_clusters_precond_and_solve(rr, kind):
    """Clusters of 700 and 300 features (several 256-member chunks of the
    restriction sum) beside small ones: the preconditioner and a fixed-count
    solve against the oracle.  The V(1,1) cycle's second row pass goes
    through the label table (X e2 = X e1 + X P yc)."""
    P = datagen.mid_sparse()
    F = P.X.shape[1]
    rng = np.random.default_rng(31)
    perm = rng.permutation(F)
    lab = np.empty(F, dtype=np.int64)
    lab[perm[:700]] = 0
    lab[perm[700:1000]] = 1
    lab[perm[1000:]] = 2 + rng.integers(0, 198, F - 1000)
    labc, fc = kmeans.compact(lab)
    assert np.bincount(labc).max() == 700
    R = rr.Ridge(P.X, labels=lab)
    lam = 1.0
    omega = op.omega_gershgorin(P.X, lam)
    B, _ = precond.make(kind, P.X, lam, labc, fc, omega)
    r = rng.standard_normal(F)
    z = host(R.apply_precond(lam, r, kind))
    zr = B(r)
    kappa_c = np.linalg.cond(coarse.coarse_matrix(P.X, labc, fc, lam))
    assert np.linalg.norm(z - zr) <= 32 * kappa_c * 2**-52 * np.linalg.norm(zr)
    x_t, inf = krylov.solve(P.X, P.y, lam, kind, labc, fc, tol=1e-12)
    w, info = R.solve(lam, P.y, precond=kind, fixed_iters=inf.iters)
    assert np.linalg.norm(host(w) - x_t) <= 1e-10 * np.linalg.norm(x_t)


def test_singleton_clusters_one_iteration(rr):
    P = datagen.tiny_sparse()
    F = P.X.shape[1]
    R = rr.Ridge(P.X, labels=np.arange(F))
    w, info = R.solve(1.0, P.y, precond="vcycle", tol=1e-12)
    assert info["iters"] == 1
    wst = krylov.reference_solution(P.X, P.y, 1.0)
    assert np.linalg.norm(host(w) - wst) <= 1e-11 * np.linalg.norm(wst)


def test_ideal_case_one_iteration(rr):
    X, group = datagen.duplicated_columns(300, [30, 45, 20, 50, 15], 0.2, seed=8)
    R = rr.Ridge(X, n_clusters=5, seed=3)
    assert R.info["n_coarse"] == 5
    assert len(set(zip(group.tolist(), host(R.labels()).tolist()))) == 5
    y = np.random.default_rng(1).standard_normal(300)
    w, info = R.solve(0.5, y, precond="vcycle", tol=1e-12)
    assert info["iters"] == 1


# --- edge cases and errors ---------------------------------------------------------

def test_zero_rhs_and_empty_columns(rr):
    import scipy.sparse as sp
    X = datagen.zipf_binary_csr(500, 300, 5, 1.1, 4)
    keep = np.ones(300)
    keep[7] = 0.0      # an empty column
    X = sp.csr_matrix(sp.csr_matrix(X) @ sp.diags(keep))
    X.eliminate_zeros()
    X.sort_indices()
    assert X[:, 7].nnz == 0
    R = rr.Ridge(X, n_clusters=20, seed=1)
    w, info = R.solve(1.0, np.zeros(500), precond="vcycle")
    assert info["iters"] == 0 and info["status"] == 0
    assert float(torch.abs(w).max()) == 0.0
    y = np.random.default_rng(3).standard_normal(500)
    lab, fc, _, _ = kmeans.kmeans_features(X, 20, 1)
    assert np.array_equal(host(R.labels()), lab)
    x_or, inf = krylov.solve(X, y, 1.0, "vcycle", lab, fc, tol=1e-13)
    w, info = R.solve(1.0, y, precond="vcycle", fixed_iters=inf.iters)
    assert np.linalg.norm(host(w) - x_or) <= 1e-10 * np.linalg.norm(x_or)


def test_single_row_and_rhs_is_b(rr):
    import scipy.sparse as sp
    X = sp.csr_matrix(np.array([[1.0, 0.0, 1.0, 1.0]]))
    R = rr.Ridge(X)
    b = np.array([1.0, -2.0, 0.5, 3.0])
    w, info = R.solve(0.25, b, precond="jacobi", rhs_is_b=True, tol=1e-14)
    ref = np.linalg.solve(X.toarray().T @ X.toarray() + 0.25 * np.eye(4), b)
    assert np.allclose(host(w), ref, rtol=1e-12)


def test_real_valued_matrix(rr):
    import scipy.sparse as sp
    rng = np.random.default_rng(6)
    X = sp.random(800, 300, density=0.03, random_state=7, format="csr")
    X.data = rng.standard_normal(X.nnz)
    with pytest.raises(rr.RRError) as e:     # GPU k-means clusters 0/1 columns only
        rr.Ridge(X, n_clusters=30, seed=1, binary=False)
    assert e.value.status == rr.RR_ERR_UNSUPPORTED
    R = rr.Ridge(X, binary=False)
    y = rng.standard_normal(800)
    v = rng.standard_normal(300)
    assert np.allclose(host(R.apply_operator(0.7, v)), op.apply_A(X, 0.7, v), rtol=1e-12, atol=1e-12)
    x_t, inf = krylov.solve(X, y, 0.7, "jacobi", tol=1e-13)
    w, info = R.solve(0.7, y, precond="jacobi", fixed_iters=inf.iters)
    assert np.linalg.norm(host(w) - x_t) <= 1e-10 * np.linalg.norm(x_t)


def test_real_valued_operator_sliced_mid(rr):
    """The valued operator's sliced passes past one LDS slice in both
    directions: 40,000 x 30,000 (three row slices of the column pass, hot and
    cold features in the row pass) with Zipf(1.1) columns and standard-normal
    values, element by element against the oracle's operator; also with a
    few empty rows and columns and ragged sizes."""
    P = datagen.sparse_problem(40_000, 30_000, 30, seed=91)
    X = P.X.tocsr().astype(np.float64)
    rng = np.random.default_rng(92)
    X.data = rng.standard_normal(X.nnz)
    R = rr.Ridge(X, binary=False)
    for lam in (0.0, 0.3):
        v = rng.standard_normal(X.shape[1])
        got = host(R.apply_operator(lam, v))
        ref = op.apply_A(X, lam, v)
        scale = np.abs(X).T @ (np.abs(X) @ np.abs(v)) + lam * np.abs(v)
        err = np.max(np.abs(got - ref) / np.maximum(scale, 1e-300))
        print(f"[valued mid] lambda={lam}: max error / |X|^T|X||v| = {err:.2e}", flush=True)
        # both sides add up to a few thousand FP64 terms per output, in
        # different orders: the gap is a few hundred units of rounding of
        # |X|^T |X| |v| at most
        assert err <= 1e-12
    R.close()
    # ragged: rows and columns with no entries, sizes off every tile
    Y = X[:33_333, :29_999].tolil()
    Y[100:140, :] = 0.0
    Y[:, 5000:5100] = 0.0
    Y = Y.tocsr()
    Y.eliminate_zeros()
    R = rr.Ridge(Y, binary=False)
    v = rng.standard_normal(Y.shape[1])
    got = host(R.apply_operator(1.0, v))
    ref = op.apply_A(Y, 1.0, v)
    scale = np.abs(Y).T @ (np.abs(Y) @ np.abs(v)) + np.abs(v)
    assert np.max(np.abs(got - ref) / scale) <= 1e-12
    R.close()


@pytest.mark.parametrize("lam", [0.05, 0.7])
def test_real_valued_two_level(rr, lam):
    """X with negative entries: smoother weight by power iteration, coarse
    Gram built column by column from labels_in, V(1,1) and additive solves."""
    import scipy.sparse as sp
    rng = np.random.default_rng(16)
    X = sp.random(1500, 700, density=0.02, random_state=17, format="csr")
    X.data = rng.standard_normal(X.nnz)
    F = X.shape[1]
    lab = datagen.random_labels(F, 60, 5)
    labc, fc = kmeans.compact(lab)
    R = rr.Ridge(X, labels=lab, binary=False)
    assert R.info["n_coarse"] == fc
    assert np.array_equal(host(R.labels()), labc)
    K_or = coarse.coarse_gram(X, labc, fc)
    K = host(R.coarse_gram())
    assert np.abs(K - K_or).max() <= 1e-12 * np.abs(K_or).max()
    om_or = op.omega_power(X, lam, seed=0x5eed)
    om = R.smoother_weight(lam)
    assert abs(om - om_or) <= 1e-10 * om_or
    y = rng.standard_normal(1500)
    for kind in ("vcycle", "additive"):
        x_t, inf = krylov.solve(X, y, lam, kind, labc, fc, omega=om_or, tol=1e-13)
        w, info = R.solve(lam, y, precond=kind, fixed_iters=inf.iters)
        print(f"[valued {kind} lam={lam}] oracle iters={inf.iters}", flush=True)
        assert np.linalg.norm(host(w) - x_t) <= 1e-10 * np.linalg.norm(x_t)
        w, info = R.solve(lam, y, precond=kind, tol=1e-10)
        assert info["status"] == 0
        x_n, inf_n = krylov.solve(X, y, lam, kind, labc, fc, omega=om_or, tol=1e-10)
        assert abs(info["iters"] - inf_n.iters) <= 1


def test_errors(rr):
    import scipy.sparse as sp
    P = datagen.tiny_sparse()
    R = rr.Ridge(P.X, n_clusters=10, seed=1)
    with pytest.raises(rr.RRError) as e:
        R.solve(0.0, P.y)
    assert e.value.status == rr.RR_ERR_INVALID_ARG
    w, info = R.solve(1.0, P.y, precond="none", max_iter=5)
    assert info["status"] == rr.RR_ERR_NOT_CONVERGED and info["iters"] == 5
    w, info = R.solve(1.0, P.y, precond="vcycle", omega=50.0)
    assert info["status"] == rr.RR_ERR_BREAKDOWN
    # invalid CSR: column index out of range / not increasing
    rp = torch.tensor([0, 2, 3], dtype=torch.int32, device="cuda")
    ci = torch.tensor([1, 9, 0], dtype=torch.int32, device="cuda")
    with pytest.raises(rr.RRError) as e:
        rr.rr_setup(rp, ci, None, 4)
    assert e.value.status == rr.RR_ERR_INVALID_ARG
    ci = torch.tensor([2, 1, 0], dtype=torch.int32, device="cuda")
    with pytest.raises(rr.RRError) as e:
        rr.rr_setup(rp, ci, None, 4)
    assert e.value.status == rr.RR_ERR_INVALID_ARG
    with pytest.raises(rr.RRError):
        rr.Ridge(P.X, labels=np.full(500, -1))


# --- the cluster-aligned block smoother ------------------------------------------

@pytest.fixture(scope="module")
def blocked(rr):
    P = datagen.mid_sparse()
    F = P.X.shape[1]
    lab = datagen.random_labels(F, 150, 21)
    labc, fc = kmeans.compact(lab)
    R = rr.Ridge(P.X, labels=lab, block_smoother=True)
    assert np.array_equal(host(R.labels()), labc)
    print(f"[blocked] F_C={fc}", flush=True)
    return P, labc, fc, R


@pytest.mark.parametrize("kind", ["vcycle", "additive"])
def test_block_smoother_parity(rr, blocked, kind):
    """Block weight equal to the oracle's power estimate; natural stop within
    the oracle's own spread under rounding-level changes, +-1; converged and
    3-iteration iterates equal to the oracle's."""
    P, lab, fc, R = blocked
    lam = 0.5
    blocks = precond.smoother_blocks(lab, fc)
    om = precond.block_omega(P.X, lam, blocks, precond.block_inverses(P.X, lam, blocks), 0x5eed)
    w, info = R.solve(lam, P.y, precond=kind, smoother="block", tol=1e-10)
    assert abs(info["omega"] - om) <= 1e-10 * om
    # the oracle's own counts with the block inverses perturbed by <= 2 ulp
    b = op.rhs(P.X, P.y)
    rng = np.random.default_rng(1)
    its = []
    for t in range(6):
        tl = precond.TwoLevel(P.X, lam, lab, fc, om, "block")
        if t:
            tl.inv = [G * (1 + (rng.random(G.shape) - 0.5) * 4 * 2**-53) for G in tl.inv]
            tl.inv = [0.5 * (G + G.T) for G in tl.inv]
        B = tl.vcycle if kind == "vcycle" else tl.additive
        _, inf = krylov.pcg(lambda v: op.apply_A(P.X, lam, v), b, B, tol=1e-10)
        its.append(inf.iters)
    print(f"[block {kind}] gpu {info['iters']} its, oracle {min(its)}..{max(its)}", flush=True)
    assert min(its) - 1 <= info["iters"] <= max(its) + 1
    x13, inf13 = krylov.solve(P.X, P.y, lam, kind, lab, fc, omega=om, tol=1e-13, smoother="block")
    w, info = R.solve(lam, P.y, precond=kind, smoother="block", fixed_iters=inf13.iters)
    assert np.linalg.norm(host(w) - x13) <= 1e-10 * np.linalg.norm(x13)
    x3, _ = krylov.solve(P.X, P.y, lam, kind, lab, fc, omega=om, fixed_iters=3, smoother="block")
    w, info = R.solve(lam, P.y, precond=kind, smoother="block", fixed_iters=3)
    assert np.linalg.norm(host(w) - x3) <= 1e-11 * np.linalg.norm(x3)


def test_block_smoother_fcg_and_options(rr, blocked):
    P, lab, fc, R = blocked
    w, info = R.solve(0.5, P.y, precond="vcycle", smoother="block", krylov="fcg", fcg_m=2, tol=1e-10)
    assert info["status"] == 0
    with pytest.raises(rr.RRError) as e:           # the block smoother belongs to two-level forms
        R.solve(0.5, P.y, precond="jacobi", smoother="block")
    assert e.value.status == rr.RR_ERR_INVALID_ARG
    R2 = rr.Ridge(P.X, labels=lab)                  # no blocks built
    with pytest.raises(rr.RRError) as e:
        R2.solve(0.5, P.y, precond="vcycle", smoother="block")
    assert e.value.status == rr.RR_ERR_INVALID_ARG
    R2.close()


def test_block_smoother_valued_x(rr):
    import scipy.sparse as sp
    rng = np.random.default_rng(26)
    X = sp.random(1500, 700, density=0.02, random_state=27, format="csr")
    X.data = rng.standard_normal(X.nnz)
    lab = datagen.random_labels(700, 40, 8)
    labc, fc = kmeans.compact(lab)
    R = rr.Ridge(X, labels=lab, binary=False, block_smoother=True)
    y = rng.standard_normal(1500)
    lam = 0.3
    blocks = precond.smoother_blocks(labc, fc)
    om = precond.block_omega(X, lam, blocks, precond.block_inverses(X, lam, blocks), 0x5eed)
    x13, inf13 = krylov.solve(X, y, lam, "vcycle", labc, fc, omega=om, tol=1e-13, smoother="block")
    w, info = R.solve(lam, y, precond="vcycle", smoother="block", fixed_iters=inf13.iters)
    assert abs(info["omega"] - om) <= 1e-10 * om
    assert np.linalg.norm(host(w) - x13) <= 1e-10 * np.linalg.norm(x13)
    R.close()


# --- TLFCG: flexible CG with the CG rougher (the paper's configuration) -----------

@pytest.mark.parametrize("steps", [2, 1, 3])
def test_tlfcg_parity(rr, clustered, steps):
    """Early iterates equal to the oracle's to rounding; converged iterates
    within 1e-10; the natural stop within 2 iterations or 5 % of the oracle's
    count (a nonlinear preconditioner inside flexible CG amplifies rounding
    differences more than a fixed one)."""
    name, P, R, (lab, fc, it, centres) = clustered
    lam = 1.0
    x3, _ = krylov.solve_tlfcg(P.X, P.y, lam, lab, fc, steps=steps, fixed_iters=3)
    w, info = R.solve(lam, P.y, precond="rougher", krylov="fcg", fcg_m=1, rougher_steps=steps,
                      fixed_iters=3)
    assert info["iters"] == 3
    assert np.linalg.norm(host(w) - x3) <= 1e-10 * np.linalg.norm(x3)
    if steps != 2:
        return
    x13, inf13 = krylov.solve_tlfcg(P.X, P.y, lam, lab, fc, tol=1e-13)
    w, info = R.solve(lam, P.y, precond="rougher", krylov="fcg", fcg_m=1, fixed_iters=inf13.iters)
    assert np.linalg.norm(host(w) - x13) <= 1e-10 * np.linalg.norm(x13)
    _, inf = krylov.solve_tlfcg(P.X, P.y, lam, lab, fc, tol=1e-10)
    w, info = R.solve(lam, P.y, precond="rougher", krylov="fcg", fcg_m=1, tol=1e-10)
    print(f"[tlfcg {name}] gpu {info['iters']} its, oracle {inf.iters}; "
          f"operator applications {info['op_applies']}", flush=True)
    assert info["status"] == 0 and info["true_relres"] <= 1e-9
    assert abs(info["iters"] - inf.iters) <= max(2, inf.iters // 20)


def test_tlfcg_jacobi_rougher(rr, clustered):
    """The Jacobi-preconditioned rougher: early and converged iterates equal
    to the oracle's."""
    name, P, R, (lab, fc, it, centres) = clustered
    lam = 1.0
    x3, _ = krylov.solve_tlfcg(P.X, P.y, lam, lab, fc, fixed_iters=3, jacobi=True)
    w, info = R.solve(lam, P.y, precond="rougher", krylov="fcg", fcg_m=1, rougher_jacobi=True,
                      fixed_iters=3)
    assert np.linalg.norm(host(w) - x3) <= 1e-10 * np.linalg.norm(x3)
    x13, inf13 = krylov.solve_tlfcg(P.X, P.y, lam, lab, fc, tol=1e-13, jacobi=True)
    w, info = R.solve(lam, P.y, precond="rougher", krylov="fcg", fcg_m=1, rougher_jacobi=True,
                      fixed_iters=inf13.iters)
    print(f"[tlfcg jacobi {name}] oracle {inf13.iters} its to 1e-13", flush=True)
    assert np.linalg.norm(host(w) - x13) <= 1e-10 * np.linalg.norm(x13)


def test_tlfcg_needs_flexible_cg(rr, clustered):
    name, P, R, _ = clustered
    with pytest.raises(rr.RRError) as e:
        R.solve(1.0, P.y, precond="rougher")
    assert e.value.status == rr.RR_ERR_INVALID_ARG


def test_vcycle_restriction_from_the_row_pass(rr):
    """The V(1,1) cycle's restriction P^T (r - A e1), formed without the
    fine-level residual as P^T (r - lam e1) - (X P)^T (X e1): a cluster of
    14 dense features (hundreds of X P column-pass pieces, summed by piece
    items), a cluster of 2000 members (finished from chunk sums), 20 small
    clusters and one whose five features have no entries.  B r and the
    converged solve against the oracle."""
    import scipy.sparse as sp
    rng = np.random.default_rng(61)
    N, F, nd = 40_000, 3000, 14
    rd, cd = np.nonzero(rng.random((N, nd)) < 0.9)
    rs = np.repeat(np.arange(N), 10)
    cs = rng.integers(nd, F - 5, size=rs.size)
    X = sp.csr_matrix((np.ones(rd.size + rs.size), (np.r_[rd, rs], np.r_[cd, cs])), shape=(N, F))
    X.sum_duplicates()
    X.data[:] = 1.0
    lab = np.empty(F, dtype=np.int64)
    lab[:12] = 0
    lab[12:2012] = 1
    lab[2012:F - 5] = 2 + np.arange(F - 5 - 2012) % 20
    lab[F - 5:] = 22
    fc = 23
    print(f"[xp restriction] N={N} F={F} nnz={X.nnz}", flush=True)
    lam = 1.0
    R = rr.Ridge(X, labels=lab)
    omega = op.omega_gershgorin(X, lam)
    B, _ = precond.make("vcycle", X, lam, lab, fc, omega)
    r = rng.standard_normal(F)
    z = host(R.apply_precond(lam, r, "vcycle"))
    zr = B(r)
    kappa_c = np.linalg.cond(coarse.coarse_matrix(X, lab, fc, lam))
    err = np.linalg.norm(z - zr) / np.linalg.norm(zr)
    print(f"[xp restriction] B r relative error {err:.2e}, bound {32 * kappa_c * 2**-52:.2e}", flush=True)
    assert err <= 32 * kappa_c * 2**-52
    y = rng.standard_normal(N)
    x_t, inf_t = krylov.solve(X, y, lam, "vcycle", lab, fc, tol=1e-13, max_iter=2000)
    w, info = R.solve(lam, y, precond="vcycle", fixed_iters=inf_t.iters)
    assert np.linalg.norm(host(w) - x_t) <= 1e-10 * np.linalg.norm(x_t)
    R.close()
