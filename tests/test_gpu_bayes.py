"""GPU parity of the eigen coarse solver (K = Q diag(ev) Q^T once, then
A_c(lambda)^-1 = Q diag(1/(ev + lambda)) Q^T for every lambda) and of the
noise-injection right-hand side (the Bayesian regression subsection, eq.
ni_xtx) against the CPU oracle.

Bars: Q orthogonal and Q diag(ev) Q^T = K to 1e-12 relative, ev to 1e-12 of
||K||; the preconditioner within the same kappa(A_c)-scaled bound as the
Cholesky one; fixed-count solves within 1e-10 of the oracle; the noise
right-hand side within FP64 rounding of its definition."""
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


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module", params=[201, 160])
def eig(request, rr):
    """mid-size 0/1 problem with random labels: an odd F_C (the Jacobi
    ordering's dummy index) and an even one."""
    P = datagen.mid_sparse()
    lab = datagen.random_labels(P.X.shape[1], request.param, 5)
    labc, fc = kmeans.compact(lab)
    R = rr.Ridge(P.X, labels=lab, coarse_eigen=True)
    print(f"[eigen] F_C={fc}, {R.info['eigen_sweeps']} Jacobi sweeps", flush=True)
    return P, labc, fc, R


def test_coarse_eigen_decomposition(rr, eig):
    P, labc, fc, R = eig
    assert R.info["eigen_sweeps"] >= 1
    Q, ev = (host(t) for t in R.coarse_eigen())
    K = coarse.coarse_gram(P.X, labc, fc)
    nK = np.linalg.norm(K)
    assert np.linalg.norm(Q.T @ Q - np.eye(fc)) <= 1e-12 * np.sqrt(fc)
    assert np.linalg.norm((Q * ev) @ Q.T - K) <= 1e-12 * nK
    ev_ref, _ = coarse.coarse_eigen(K)
    assert np.max(np.abs(np.sort(ev) - ev_ref)) <= 1e-12 * nK


def test_eigen_coarse_inverse_and_factor_options(rr, eig):
    P, labc, fc, R = eig
    K = coarse.coarse_gram(P.X, labc, fc)
    for lam in (1e-2, 1.0, 100.0):
        Ai = torch.empty(fc * fc, dtype=torch.float64, device="cuda")
        rr.rr_coarse_factor(R.h, lam, None, Ai)
        ref = np.linalg.inv(K + lam * np.eye(fc))
        kappa = np.linalg.cond(K + lam * np.eye(fc))
        assert np.linalg.norm(host(Ai).reshape(fc, fc) - ref) <= 64 * kappa * 2**-52 * np.linalg.norm(ref)
    with pytest.raises(rr.RRError):
        R.coarse_factor(1.0)   # asks for L, which the eigen form does not make


@pytest.mark.parametrize("kind", ["vcycle", "additive"])
def test_eigen_precond_and_solve_parity(rr, eig, kind):
    P, labc, fc, R = eig
    rng = np.random.default_rng(3)
    for lam in (1e-2, 1.0, 100.0):
        omega = op.omega_gershgorin(P.X, lam)
        B, _ = precond.make(kind, P.X, lam, labc, fc, omega)
        r = rng.standard_normal(P.X.shape[1])
        z = host(R.apply_precond(lam, r, kind))
        zr = B(r)
        kappa_c = np.linalg.cond(coarse.coarse_matrix(P.X, labc, fc, lam))
        assert np.linalg.norm(z - zr) <= 64 * kappa_c * 2**-52 * np.linalg.norm(zr), lam
    lam = 0.3
    x_t, inf = krylov.solve(P.X, P.y, lam, kind, labc, fc, tol=1e-12)
    w, info = R.solve(lam, P.y, precond=kind, fixed_iters=inf.iters)
    assert np.linalg.norm(host(w) - x_t) <= 1e-10 * np.linalg.norm(x_t)


def test_noise_rhs_and_sample(rr, eig):
    P, labc, fc, R = eig
    N, F = P.X.shape
    rng = np.random.default_rng(11)
    xi1, xi2 = rng.standard_normal(N), rng.standard_normal(F)
    tau, lam = 3.0, 0.7
    b = host(R.noise_rhs(tau, lam, P.y, xi1, xi2))
    want = op.noise_rhs(P.X, P.y, tau, lam, xi1, xi2)
    scale = np.abs(P.X.T) @ (np.abs(P.y) + np.abs(xi1) / np.sqrt(tau)) + np.sqrt(lam) / tau * np.abs(xi2)
    assert np.all(np.abs(b - want) <= 64 * 2**-52 * scale)
    # the sample: (X^T X + (lam / tau) I) w = b, solved to the oracle's answer
    beta = lam / tau
    w, info = R.solve(beta, b, rhs_is_b=True, precond="vcycle", tol=1e-12)
    assert info["status"] == 0
    A = lambda v: op.apply_A(P.X, beta, v)
    ws, _ = krylov.pcg(A, want, lambda r: r / op.jacobi_diagonal(P.X, beta), tol=1e-13, max_iter=20000)
    assert np.linalg.norm(host(w) - ws) <= 1e-9 * np.linalg.norm(ws)
