"""Pins for the oracle's generator, operator, smoother weight and coarse
level: checked against published test vectors, brute force, closed forms and
invariants, never against the oracle itself."""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import datagen
from oracle import SplitMix64, coarse, operator as op
from tests.conftest import read_golden


def test_splitmix64_published_vectors():
    rows = read_golden("splitmix64.txt")
    assert rows[0] == ["seed", "1234567"]
    r = SplitMix64(1234567)
    for tok in rows[1:6]:
        assert r.next() == int(tok[0])


def test_splitmix64_unit_draws_follow_the_published_outputs():
    """next_unit() is the top 53 bits of next() over 2^53: on the published
    seed it must give exactly those fractions (Fraction arithmetic, no
    rounding), and over many draws it must look uniform on [0, 1)."""
    rows = read_golden("splitmix64.txt")
    r = SplitMix64(int(rows[0][1]))
    for tok in rows[1:6]:
        u = r.next_unit()
        assert Fraction(u) == Fraction(int(tok[0]) >> 11, 1 << 53)
        assert 0.0 <= u < 1.0
    # chi-square of 5 equal buckets over 100,000 draws: 4 degrees of
    # freedom, P(chi2 > 18.47) = 0.001
    r = SplitMix64(987654321)
    n = 100000
    counts = [0] * 5
    for _ in range(n):
        counts[int(r.next_unit() * 5)] += 1
    chi2 = sum((c - n / 5) ** 2 / (n / 5) for c in counts)
    assert chi2 < 18.47, counts


def _tiny_binary(seed, n=40, f=17, m=4):
    return datagen.zipf_binary_csr(n, f, m, 1.1, seed)


def test_operator_exact_on_integers_brute_force():
    """Binary X, integer v, integer lam: every intermediate is an integer,
    so A v must equal a Python-int brute force exactly."""
    X = _tiny_binary(1)
    rng = np.random.default_rng(0)
    v = rng.integers(-50, 50, size=X.shape[1]).astype(np.float64)
    lam = 3.0
    Xd = X.toarray().astype(int)
    Xv = [sum(int(Xd[i, j]) * int(v[j]) for j in range(X.shape[1])) for i in range(X.shape[0])]
    ref = [sum(int(Xd[i, j]) * Xv[i] for i in range(X.shape[0])) + 3 * int(v[j])
           for j in range(X.shape[1])]
    got = op.apply_A(X, lam, v)
    assert [int(g) for g in got] == ref
    assert np.all(got == np.asarray(ref, dtype=np.float64))


def test_operator_random_vector_fsum():
    X = _tiny_binary(2)
    rng = np.random.default_rng(1)
    v = rng.standard_normal(X.shape[1])
    lam = 0.37
    Xd = X.toarray()
    u = [math.fsum(Xd[i, j] * v[j] for j in range(X.shape[1])) for i in range(X.shape[0])]
    ref = np.array([math.fsum([Xd[i, j] * u[i] for i in range(X.shape[0])] + [lam * v[j]])
                    for j in range(X.shape[1])])
    got = op.apply_A(X, lam, v)
    scale = np.abs(Xd).T @ (np.abs(Xd) @ np.abs(v)) + lam * np.abs(v)
    assert np.all(np.abs(got - ref) <= 64 * np.finfo(float).eps * scale)


def test_rhs_and_diagonal():
    X = _tiny_binary(3)
    Xd = X.toarray()
    y = np.arange(X.shape[0], dtype=float) - 7
    assert np.allclose(op.rhs(X, y), Xd.T @ y, rtol=0, atol=1e-12)
    assert np.array_equal(op.jacobi_diagonal(X, 2.0), np.diag(Xd.T @ Xd) + 2.0)


@pytest.mark.parametrize("lam", [1e-2, 1.0, 100.0])
def test_gershgorin_weight_bounds_spectrum(lam):
    X = _tiny_binary(4, n=60, f=25, m=6)
    Xd = X.toarray()
    A = Xd.T @ Xd + lam * np.eye(X.shape[1])
    D = np.diag(A)
    rho = sla.eigh(A, np.diag(D), eigvals_only=True).max()   # rho(D^-1 A)
    w = op.omega_gershgorin(X, lam)
    assert 1.0 / w >= rho * (1 - 1e-12)
    assert w * rho < 2.0


def test_power_weight_keeps_smoother_convergent():
    rng = np.random.default_rng(5)
    Xd = rng.standard_normal((50, 20))
    lam = 0.1
    A = Xd.T @ Xd + lam * np.eye(20)
    rho = sla.eigh(A, np.diag(np.diag(A)), eigvals_only=True).max()
    w = op.omega_power(Xd, lam, seed=9)
    assert w * rho < 2.0
    assert w * rho > 0.5          # not uselessly small: estimate within 2x
    with pytest.raises(ValueError):
        op.omega_gershgorin(Xd, lam)


def test_prolongation_is_orthonormal():
    labels = np.array([0, 2, 1, 2, 2, 0, 3, 1, 2])
    P = coarse.prolongation(labels, 4)
    PtP = (P.T @ P).toarray()
    off = PtP - np.diag(np.diag(PtP))
    assert np.all(off == 0)
    assert np.all(np.abs(np.diag(PtP) - 1.0) <= 2 * np.finfo(float).eps)


def test_averaging_restriction_gram_golden():
    rows = read_golden("averaging_restriction.txt")
    sizes = [int(t) for t in rows[0][1:]]
    diag = [float(t) for t in rows[1][1:]]
    labels = np.repeat(np.arange(len(sizes)), sizes)
    Pt = coarse.averaging_restriction(labels, len(sizes))
    G = (Pt @ Pt.T).toarray()
    assert np.allclose(G, np.diag(diag), rtol=1e-15, atol=0)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_galerkin_identity(seed):
    """A_c = P^T (X^T X + lam I) P, formed densely from its definition."""
    X = _tiny_binary(10 + seed, n=80, f=30, m=5)
    labels = datagen.random_labels(30, 7, seed)
    lam = 0.5
    Xd = X.toarray()
    P = coarse.prolongation(labels, 7).toarray()
    ref = P.T @ (Xd.T @ Xd + lam * np.eye(30)) @ P
    Ac = coarse.coarse_matrix(X, labels, 7, lam)
    assert np.max(np.abs(Ac - ref)) <= 1e-13 * np.max(np.abs(ref))
    # binary X: sqrt(n_s n_t) K_st is the integer S^T S with S = X P_u
    n = coarse.cluster_sizes(labels, 7)
    K = coarse.coarse_gram(X, labels, 7)
    Pu = np.zeros((30, 7), dtype=np.int64)
    Pu[np.arange(30), labels] = 1
    S = X.toarray().astype(np.int64) @ Pu
    StS = S.T @ S
    assert np.allclose(K * np.sqrt(np.outer(n, n)), StS, rtol=1e-14, atol=0)


def test_galerkin_identity_real_valued():
    rng = np.random.default_rng(12)
    X = sp.random(70, 25, density=0.2, random_state=3, format="csr")
    X.data = rng.standard_normal(X.nnz)
    labels = datagen.random_labels(25, 6, 1)
    Xd = X.toarray()
    P = coarse.prolongation(labels, 6).toarray()
    ref = P.T @ (Xd.T @ Xd + 0.3 * np.eye(25)) @ P
    Ac = coarse.coarse_matrix(X, labels, 6, 0.3)
    assert np.max(np.abs(Ac - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_cholesky_factor():
    X = _tiny_binary(20, n=90, f=40, m=5)
    labels = datagen.random_labels(40, 9, 3)
    Ac = coarse.coarse_matrix(X, labels, 9, 0.1)
    L = coarse.cholesky(Ac)
    assert np.allclose(L, np.tril(L))
    assert np.linalg.norm(L @ L.T - Ac) <= 1e-14 * np.linalg.norm(Ac)
    c = np.arange(9.0)
    assert np.allclose(coarse.coarse_solve(L, c), np.linalg.solve(Ac, c), rtol=1e-12)


def test_ideal_case_golden_spectrum():
    """Duplicated columns: the nonzero eigenvalues of X^T X equal those of
    K = P^T X^T X P, and match the hand-derived closed form 5 -/+ sqrt(7)."""
    rows = read_golden("ideal_case.txt")
    x1 = np.array([float(t) for t in rows[0][1:]])
    x2 = np.array([float(t) for t in rows[1][1:]])
    n1, n2 = (int(t) for t in rows[2][1:])
    Kg = np.array([float(t) for t in rows[3][1:]]).reshape(2, 2)
    eig = np.array([float(t) for t in rows[4][1:]])
    Xd = np.column_stack([x1] * n1 + [x2] * n2)
    labels = np.array([0] * n1 + [1] * n2)
    K = coarse.coarse_gram(sp.csr_matrix(Xd), labels, 2)
    assert np.allclose(K, Kg, rtol=1e-15, atol=1e-15)
    ev = np.linalg.eigvalsh(Xd.T @ Xd)
    nz = np.sort(ev[np.abs(ev) > 1e-9])
    assert np.allclose(nz, eig, rtol=1e-14)
    assert np.allclose(np.linalg.eigvalsh(K), eig, rtol=1e-14)
    # the printed scaling x_s^T x_t / sqrt(n_s n_t) does not reproduce it
    wrong = np.array([[x1 @ x1 / n1, x1 @ x2 / math.sqrt(n1 * n2)],
                      [x1 @ x2 / math.sqrt(n1 * n2), x2 @ x2 / n2]])
    assert not np.allclose(np.linalg.eigvalsh(wrong), eig)


def test_exact_argmin_against_fractions():
    from oracle.kmeans import exact_argmin
    rng = np.random.default_rng(7)
    for trial in range(20):
        F, k = 30, 6
        den = rng.integers(1, 6, size=k) ** 2
        num = rng.integers(-40, 40, size=(F, k))
        active = rng.random(k) > 0.2
        active[rng.integers(k)] = True
        got = exact_argmin(num, den, active)
        for j in range(F):
            best = None
            for s in range(k):
                if not active[s]:
                    continue
                v = Fraction(int(num[j, s]), int(den[s]))
                if best is None or v < best[0]:
                    best = (v, s)
            assert got[j] == best[1]
    # huge values take the Python-int path
    num = np.array([[3 * 10**12, 3 * 10**12 - 1]], dtype=np.int64)
    den = np.array([10**10, 10**10], dtype=np.int64)
    assert exact_argmin(num, den, np.array([True, True]))[0] == 1


def test_bf16_round_ties_and_specials():
    """Round to nearest, ties to even, at 8 significant bits; FP32 range."""
    v = np.array([1.0, 1 + 2**-8, 1 + 3 * 2**-8, 1 + 2**-8 + 2**-20, -(1 + 3 * 2**-8),
                  65504.0, 0.0, np.inf, -np.inf, 2.0**100 * (1 + 2**-9)])
    want = np.array([1.0, 1.0, 1 + 2**-6, 1 + 2**-7, -(1 + 2**-6), 65536.0, 0.0, np.inf,
                     -np.inf, 2.0**100])
    assert np.array_equal(op.bf16_round(v), want)
    # every BF16 value is a fixed point; neighbours 2^-7 apart at 1
    r = np.random.default_rng(3).standard_normal(1000)
    b = op.bf16_round(r)
    assert np.array_equal(op.bf16_round(b), b)
    assert np.all(np.abs(b - r) <= 2.0**-8 * np.abs(r) * (1 + 2**-20))


def test_bf16_operator_bound_covers_a_perturbed_sum():
    """The bound admits the FP32-summed operator on random data and is tight
    enough to reject a transposed operand."""
    rng = np.random.default_rng(4)
    X = rng.standard_normal((60, 20)).astype(np.float32).astype(np.float64)
    V = rng.standard_normal((20, 3))
    Q = op.apply_A_bf16(X, 0.5, V)
    B = op.apply_A_bf16_bound(X, V)
    Xb = op.bf16_round(X)
    U32 = (Xb.astype(np.float32) @ op.bf16_round(V).astype(np.float32)).astype(np.float64)
    Q32 = (Xb.T.astype(np.float32) @ op.bf16_round(U32).astype(np.float32)).astype(np.float64) + 0.5 * V
    assert np.all(np.abs(Q32 - Q) <= B)
    Xs = X.copy()
    Xs[:, [0, 1]] = Xs[:, [1, 0]]                # a swapped pair of columns
    assert np.any(np.abs(op.apply_A_bf16(Xs, 0.5, V) - Q) > B)
    assert B.max() < 0.1 * np.abs(Q).max()


def test_f32_operator_bound_covers_a_perturbed_sum():
    """The FP32 bound admits an FP32-summed operator and rejects a swapped
    pair of columns."""
    rng = np.random.default_rng(5)
    X = rng.standard_normal((300, 40)).astype(np.float32).astype(np.float64)
    V = rng.standard_normal((40, 3))
    Q = op.apply_A_f32(X, 0.5, V)
    B = op.apply_A_f32_bound(X, V)
    U32 = (X.astype(np.float32) @ V.astype(np.float32))
    Q32 = (X.T.astype(np.float32) @ U32).astype(np.float64) + 0.5 * V
    assert np.all(np.abs(Q32 - Q) <= B)
    Xs = X.copy()
    Xs[:, [0, 1]] = Xs[:, [1, 0]]
    assert np.any(np.abs(op.apply_A_f32(Xs, 0.5, V) - Q) > B)
    assert B.max() < 1e-3 * np.abs(Q).max()


# --- the eigen coarse solver and the noise-injection sampler ------------------

def test_eigen_coarse_inverse_closed_form_and_svd():
    """A_c(lam)^-1 from K = Q diag(ev) Q^T equals inv(K + lam I) at several
    lam, and equals the SVD form V diag(1/(s^2 + lam)) V^T built from the
    right singular vectors of X_c = X P (the paper's coarse solver for
    Bayesian regression)."""
    P = datagen.sparse_problem(400, 90, 8, seed=21)
    lab = datagen.random_labels(90, 12, 4)
    labc = np.unique(lab, return_inverse=True)[1]
    fc = int(labc.max()) + 1
    K = coarse.coarse_gram(P.X, labc, fc)
    ev, Q = coarse.coarse_eigen(K)
    assert np.allclose(Q.T @ Q, np.eye(fc), atol=1e-13)
    assert np.linalg.norm(Q @ np.diag(ev) @ Q.T - K) <= 1e-13 * np.linalg.norm(K)
    Xc = (P.X @ coarse.prolongation(labc, fc)).toarray()
    _, s, Vt = np.linalg.svd(Xc, full_matrices=False)
    for lam in (1e-2, 1.0, 37.0):
        Ai = coarse.eigen_coarse_inverse(ev, Q, lam)
        ref = np.linalg.inv(K + lam * np.eye(fc))
        assert np.linalg.norm(Ai - ref) <= 1e-11 * np.linalg.norm(ref)
        svd = (Vt.T / (s**2 + lam)) @ Vt
        assert np.linalg.norm(Ai - svd) <= 1e-11 * np.linalg.norm(ref)


def test_noise_rhs_reduces_to_rhs_and_is_linear():
    P = datagen.sparse_problem(300, 40, 6, seed=23)
    rng = np.random.default_rng(1)
    xi1, xi2 = rng.standard_normal(300), rng.standard_normal(40)
    z1, z2 = np.zeros(300), np.zeros(40)
    assert np.array_equal(op.noise_rhs(P.X, P.y, 2.0, 3.0, z1, z2), op.rhs(P.X, P.y))
    # b - X^T y = X^T xi1 / sqrt(tau) + sqrt(lam) / tau xi2, term by term
    b = op.noise_rhs(P.X, P.y, 4.0, 9.0, xi1, xi2)
    want = op.rhs(P.X, P.y) + (P.X.T @ xi1) / 2.0 + (3.0 / 4.0) * xi2
    assert np.allclose(b, want, rtol=1e-14, atol=1e-13)


def test_noise_injection_samples_the_posterior():
    """Solving (X^T X + (lam/tau) I) w = X^T (y + e1) + e2 / tau draws w from
    N((X^T X + beta I)^-1 X^T y, ((X^T X + beta I) tau)^-1) with beta =
    lam / tau (the Bayesian regression subsection): the sample mean and
    covariance of 40,000 draws match to within their sampling error."""
    rng = np.random.default_rng(7)
    N, F, tau, lam = 60, 5, 2.5, 4.0
    X = rng.standard_normal((N, F))
    y = rng.standard_normal(N)
    M = X.T @ X + (lam / tau) * np.eye(F)
    S = 40_000
    xi1 = rng.standard_normal((S, N))
    xi2 = rng.standard_normal((S, F))
    B = np.stack([op.noise_rhs(X, y, tau, lam, xi1[i], xi2[i]) for i in range(S)])
    W = np.linalg.solve(M, B.T).T
    mean_ref = np.linalg.solve(M, X.T @ y)
    cov_ref = np.linalg.inv(M * tau)
    sd = np.sqrt(np.diag(cov_ref))
    assert np.all(np.abs(W.mean(0) - mean_ref) <= 5 * sd / np.sqrt(S))
    C = np.cov(W.T)
    # sampling error of a covariance entry: about sqrt((s_ii s_jj + s_ij^2) / S)
    err = np.sqrt((np.outer(np.diag(cov_ref), np.diag(cov_ref)) + cov_ref**2) / S)
    assert np.all(np.abs(C - cov_ref) <= 5 * err)
    # a mistaken scale (e1 with variance 1/tau^2, or e2 / sqrt(tau)) is ruled out
    bad = np.linalg.inv(M * tau * tau)
    assert np.any(np.abs(C - bad) > 5 * err)


def test_weighted_operator_is_the_logistic_hessian():
    """For L2-regularized logistic regression f(w) = sum_i log(1 + e^{z_i})
    - t_i z_i + beta ||w||^2 / 2 with z = X w, the Hessian is X^T D X + beta I
    with D = diag(p (1 - p)), p = sigma(z): apply_A of weighted_rows(X, d)
    equals central differences of the analytic gradient X^T (p - t) + beta w."""
    P = datagen.sparse_problem(500, 60, 7, seed=29)
    X = P.X
    rng = np.random.default_rng(3)
    t = (rng.random(500) < 0.4).astype(np.float64)
    w = 0.3 * rng.standard_normal(60)
    beta = 0.7
    grad = lambda w: X.T @ (1.0 / (1.0 + np.exp(-(X @ w))) - t) + beta * w
    p = 1.0 / (1.0 + np.exp(-(X @ w)))
    Xd = op.weighted_rows(X, p * (1.0 - p))
    for _ in range(3):
        v = rng.standard_normal(60)
        eps = 1e-5
        fd = (grad(w + eps * v) - grad(w - eps * v)) / (2 * eps)
        hv = op.apply_A(Xd, beta, v)
        assert np.linalg.norm(hv - fd) <= 1e-7 * np.linalg.norm(hv)
    with pytest.raises(ValueError):
        op.weighted_rows(X, -np.ones(500))
