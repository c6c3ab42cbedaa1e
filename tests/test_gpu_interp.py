"""GPU parity of least-squares interpolation (rr_set_interpolation) against
the CPU oracle: the weights, the Galerkin coarse matrix with its P^T P term,
the two-level preconditioner and solves, and the error paths."""
import numpy as np
import pytest

import datagen
from oracle import interp, kmeans, krylov, leader, precond
from oracle.operator import omega_gershgorin

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


def principal(X, K):
    G = (X.T @ X).toarray()
    ev, Q = np.linalg.eigh(G)
    return np.ascontiguousarray(Q[:, ::-1][:, :K])


CASES = {
    "tiny": lambda: datagen.tiny_sparse(),
    "ragged": lambda: datagen.sparse_problem(3001, 1237, 7, seed=77),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("agg", ["lf", "kmeans"])
def test_weights_and_coarse_matrix(rr, name, agg):
    P = CASES[name]()
    X = P.X
    F = X.shape[1]
    if agg == "lf":
        lab, fc, _ = leader.leader_follower(X, 3.0)
        R = rr.Ridge(X, lf_tolerance=3.0)
    else:
        lab, fc, _, _ = kmeans.kmeans_features(X, 24, 3)
        R = rr.Ridge(X, n_clusters=24, seed=3)
    assert np.array_equal(host(R.labels()), lab)
    V = principal(X, 5)
    beta = 0.5
    eta = interp.prototype_energies(X, V, beta)
    p_or = interp.ls_weights(V, eta, lab, fc, interp.representatives(lab, fc))
    print(f"[ls {name} {agg}] F={F} F_C={fc}", flush=True)
    p = host(R.set_interpolation(V, beta))
    assert np.allclose(p, p_or, rtol=1e-10, atol=1e-12 * np.abs(p_or).max())
    Pm = interp.ls_prolongation(lab, fc, p_or)
    lam = 0.7
    Ac = interp.galerkin_coarse(X, Pm, lam)
    K = host(R.coarse_gram())
    assert np.allclose(K, Ac - lam * (Pm.T @ Pm).toarray(), rtol=1e-10, atol=1e-11 * np.abs(Ac).max())
    _, Ainv = R.coarse_factor(lam)
    ref = np.linalg.inv(Ac)
    assert np.allclose(host(Ainv), ref, rtol=1e-8, atol=1e-9 * np.abs(ref).max())
    R.close()


def test_precond_and_solves(rr):
    Pb = datagen.sparse_problem(3001, 1237, 7, seed=77)
    X, y = Pb.X, Pb.y
    lab, fc, _ = leader.leader_follower(X, 3.0)
    V = principal(X, 6)
    lam = 0.5
    eta = interp.prototype_energies(X, V, lam)
    p = interp.ls_weights(V, eta, lab, fc, interp.representatives(lab, fc))
    Pm = interp.ls_prolongation(lab, fc, p)
    R = rr.Ridge(X, lf_tolerance=3.0)
    R.set_interpolation(V, lam)
    om = omega_gershgorin(X, lam)
    tl = precond.TwoLevel(X, lam, lab, fc, om, P=Pm)
    r = np.random.default_rng(11).standard_normal(X.shape[1])
    for kind, fn in (("vcycle", tl.vcycle), ("additive", tl.additive)):
        z = host(R.apply_precond(lam, r, precond=kind, omega=om))
        ref = fn(r)
        assert np.linalg.norm(z - ref) <= 1e-11 * np.linalg.norm(ref), kind
    for kind in ("vcycle", "additive"):
        x_or, inf = krylov.solve(X, y, lam, kind, lab, fc, tol=1e-12, P=Pm)
        w, info = R.solve(lam, y, precond=kind, fixed_iters=inf.iters)
        assert np.linalg.norm(host(w) - x_or) <= 1e-10 * np.linalg.norm(x_or), kind
        w, info = R.solve(lam, y, precond=kind, tol=1e-10)
        assert info["iters"] <= inf.iters and info["true_relres"] <= 2e-10, kind
    R.close()


def test_tlfcg_with_least_squares_interpolation(rr):
    """The paper's configuration (flexible CG, two CG pre-smoothing steps)
    on the least-squares prolongation: early iterates to rounding, and the
    natural stop within 2 iterations or 5 % of the oracle's count."""
    Pb = datagen.sparse_problem(3001, 1237, 7, seed=77)
    X, y = Pb.X, Pb.y
    lab, fc, _ = leader.leader_follower(X, 3.0)
    V = principal(X, 4)
    lam = 1.0
    eta = interp.prototype_energies(X, V, lam)
    Pm = interp.ls_prolongation(lab, fc, interp.ls_weights(V, eta, lab, fc,
                                                            interp.representatives(lab, fc)))
    R = rr.Ridge(X, lf_tolerance=3.0)
    R.set_interpolation(V, lam)
    x3, _ = krylov.solve_tlfcg(X, y, lam, lab, fc, fixed_iters=3, P=Pm)
    w, info = R.solve(lam, y, precond="rougher", krylov="fcg", fcg_m=1, fixed_iters=3)
    assert np.linalg.norm(host(w) - x3) <= 1e-10 * np.linalg.norm(x3)
    _, inf = krylov.solve_tlfcg(X, y, lam, lab, fc, tol=1e-10, P=Pm)
    w, info = R.solve(lam, y, precond="rougher", krylov="fcg", fcg_m=1, tol=1e-10)
    assert info["status"] == 0 and info["true_relres"] <= 1e-9
    assert abs(info["iters"] - inf.iters) <= max(2, inf.iters // 20)
    R.close()


def test_graph_replays_equal_eager(rr):
    """Captured iterations with the least-squares restriction and
    prolongation replay bitwise equal to eager runs; changing the
    interpolation drops the captured graphs."""
    P = datagen.sparse_problem(3001, 1237, 7, seed=77)
    R = rr.Ridge(P.X, lf_tolerance=3.0)
    R.set_interpolation(principal(P.X, 4), 1.0)
    for rep in range(3):
        for lam in (0.1, 1.0):
            we, ie = R.solve(lam, P.y, precond="vcycle", tol=1e-10, chunk=4)
            wg, ig = R.solve(lam, P.y, precond="vcycle", tol=1e-10, chunk=4, graph=True)
            assert ie["iters"] == ig["iters"] and ie["status"] == ig["status"] == 0
            assert np.array_equal(host(we), host(wg)), (rep, lam)
            R.apply_operator(lam, np.ones(P.X.shape[1]))
    R.set_interpolation(None)
    we, ie = R.solve(1.0, P.y, precond="vcycle", tol=1e-10, chunk=4)
    wg, ig = R.solve(1.0, P.y, precond="vcycle", tol=1e-10, chunk=4, graph=True)
    assert np.array_equal(host(we), host(wg))
    R.close()


def test_batched_lambdas_on_one_handle(rr):
    """Several lambdas in one rr_solve_batched call (one work set each, with
    its own restriction buffers) equal one rr_solve after another."""
    P = datagen.sparse_problem(3001, 1237, 7, seed=77)
    R = rr.Ridge(P.X, lf_tolerance=3.0)
    R.set_interpolation(principal(P.X, 4), 1.0)
    lams = [0.1, 1.0, 10.0]
    y = torch.as_tensor(P.y, dtype=torch.float64, device="cuda")
    ws = [torch.empty(P.X.shape[1], dtype=torch.float64, device="cuda") for _ in lams]
    st, infos = rr.rr_solve_batched([R.h] * len(lams), lams, [y] * len(lams), ws, tol=1e-10,
                                    precond="vcycle")
    assert st == 0
    for lam, w, inf in zip(lams, ws, infos):
        w1, inf1 = R.solve(lam, P.y, precond="vcycle", tol=1e-10)
        assert inf["status"] == 0 and inf["iters"] == inf1["iters"]
        assert np.array_equal(host(w), host(w1)), lam
    R.close()


def test_caller_representatives_and_restore(rr):
    P = datagen.tiny_sparse()
    X = P.X
    lab, fc, _ = leader.leader_follower(X, 3.0)
    R = rr.Ridge(X, lf_tolerance=3.0)
    K_sa = host(R.coarse_gram()).copy()
    rng = np.random.default_rng(5)
    V = rng.standard_normal((X.shape[1], 3))
    # the last member of every cluster as its coarse feature
    rep = np.array([np.flatnonzero(lab == c)[-1] for c in range(fc)], dtype=np.int32)
    eta = interp.prototype_energies(X, V, 1.0)
    p_or = interp.ls_weights(V, eta, lab, fc, rep)
    p = host(R.set_interpolation(V, 1.0, rep=rep))
    assert np.allclose(p, p_or, rtol=1e-10, atol=1e-12 * np.abs(p_or).max())
    # a coarse feature outside its cluster is refused and the weights stay
    bad = rep.copy()
    bad[0] = int(np.flatnonzero(lab != 0)[0])
    with pytest.raises(rr.RRError):
        R.set_interpolation(V, 1.0, rep=bad)
    Vn = V.copy()
    Vn[rep[1], :] = np.nan
    with pytest.raises(rr.RRError):
        R.set_interpolation(Vn, 1.0, rep=rep)
    Pm = interp.ls_prolongation(lab, fc, p_or)
    K = host(R.coarse_gram())
    Kref = interp.galerkin_coarse(X, Pm, 0.0)
    assert np.allclose(K, Kref, rtol=1e-10, atol=1e-11 * np.abs(Kref).max())
    # unsupported with single-precision inner solves
    with pytest.raises(rr.RRError):
        R.solve(1.0, P.y, precond="vcycle", precision="f32_ir")
    # back to the adjusted square-root average: the exact integer Gram again
    assert R.set_interpolation(None) is None
    assert np.array_equal(host(R.coarse_gram()), K_sa)
    R.close()


def test_zero_energy_cluster_keeps_aggregation(rr):
    P = datagen.tiny_sparse()
    X = P.X
    lab, fc, _ = leader.leader_follower(X, 3.0)
    rep = interp.representatives(lab, fc)
    V = np.random.default_rng(8).standard_normal((X.shape[1], 2))
    big = int(np.argmax(np.bincount(lab, minlength=fc)))
    V[rep[big], :] = 0.0
    R = rr.Ridge(X, lf_tolerance=3.0)
    p = host(R.set_interpolation(V, 0.0))
    assert np.all(p[lab == big] == 1.0)
    eta = interp.prototype_energies(X, V, 0.0)
    p_or = interp.ls_weights(V, eta, lab, fc, rep)
    assert np.allclose(p, p_or, rtol=1e-10, atol=1e-12 * np.abs(p_or).max())
    R.close()


@pytest.mark.parametrize("name", list(CASES))
def test_prototypes_match_the_oracle_eigenvectors(rr, name):
    """rr_prototypes (Lanczos with full reorthogonalisation on the GPU)
    against the oracle's dense eigendecomposition of X^T X: Ritz values to
    1e-10 relative, Ritz vectors up to sign to the accuracy the spectral gap
    allows (eps ||X^T X|| / gap), and the eigen equation's residual."""
    P = CASES[name]()
    R = rr.Ridge(P.X, n_clusters=20, seed=1)
    K = 6
    V = torch.empty((K, P.X.shape[1]), dtype=torch.float64, device="cuda")
    ev = rr.rr_prototypes(R.h, K, V, steps=80)
    Vo, evo = interp.leading_prototypes(P.X, K + 1)
    Vg = host(V)
    G = (P.X.T @ P.X).toarray()
    print(f"[prototypes {name}] Ritz values {ev}, oracle {evo[:K]}", flush=True)
    assert np.allclose(ev, evo[:K], rtol=1e-10, atol=0)
    for k in range(K):
        gap = min(abs(evo[k] - evo[j]) for j in range(K + 1) if j != k)
        d = min(np.linalg.norm(Vg[k] - Vo[:, k]), np.linalg.norm(Vg[k] + Vo[:, k]))
        assert d <= 1e-12 * evo[0] / gap + 1e-10, (k, d, gap)
        assert np.linalg.norm(G @ Vg[k] - ev[k] * Vg[k]) <= 1e-9 * evo[0]
    # they drive rr_set_interpolation like host-made prototypes
    R2 = rr.Ridge(P.X, n_clusters=20, seed=1)
    R.set_interpolation(V.T.contiguous().cpu().numpy(), beta=1.0)
    R2.set_interpolation(Vo[:, :K], beta=1.0)
    w1, i1 = R.solve(1.0, P.y, precond="vcycle", tol=1e-10)
    w2, i2 = R2.solve(1.0, P.y, precond="vcycle", tol=1e-10)
    assert i1["status"] == 0 and abs(i1["iters"] - i2["iters"]) <= 1
    with pytest.raises(rr.RRError):
        rr.rr_prototypes(R.h, 0, V)
    with pytest.raises(rr.RRError):
        rr.rr_prototypes(R.h, K, V, steps=K - 1)
    R.close()
    R2.close()
