"""Mixed precision: FP32 inner PCG inside FP64 iterative refinement, through
the C ABI, against the FP64 oracle's solution.

Bar: the refined solution within 1e-10 relative error of the dense FP64
solution (the error is asserted per case); at least two refinement steps
(the FP32 inner solves alone cannot reach it)."""
import numpy as np
import pytest

import datagen
from oracle import krylov

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


CASES = {
    "tiny": (lambda: datagen.tiny_sparse(), 50),
    "ragged": (lambda: datagen.sparse_problem(3001, 1237, 7, seed=77), 80),
    "wide": (lambda: datagen.sparse_problem(8000, 3000, 25, seed=79), 200),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request, rr):
    gen, k = CASES[request.param]
    P = gen()
    print(f"[mixed {request.param}] N={P.X.shape[0]} F={P.X.shape[1]} nnz={P.X.nnz}", flush=True)
    return request.param, P, rr.Ridge(P.X, n_clusters=k, seed=3)


@pytest.mark.parametrize("kind", ["vcycle", "jacobi", "none"])
@pytest.mark.parametrize("lam", [1e-2, 1.0])
def test_refinement_reaches_fp64_solution(rr, case, kind, lam):
    name, P, R = case
    wst = krylov.reference_solution(P.X, P.y, lam)
    w, info = R.solve(lam, P.y, precond=kind, precision="f32_ir", tol=1e-13, max_iter=20000)
    err = np.linalg.norm(host(w) - wst) / np.linalg.norm(wst)
    print(f"[mixed {name}] {kind} lambda={lam}: {info['ir_steps']} steps, {info['iters']} inner "
          f"iterations, residual {info['relres']:.1e}, error {err:.1e}", flush=True)
    assert info["status"] == 0 and info["relres"] <= 1e-13
    assert info["ir_steps"] >= 2
    assert err <= 1e-10
    # the FP64 path to the same residual, for comparison
    w64, i64 = R.solve(lam, P.y, precond=kind, tol=1e-13, max_iter=20000)
    err64 = np.linalg.norm(host(w64) - wst) / np.linalg.norm(wst)
    assert err64 <= 1e-10


def test_inner_tolerance_trades_steps(rr, case):
    name, P, R = case
    lam = 1.0
    steps = []
    for itol in (1e-2, 1e-6):
        w, info = R.solve(lam, P.y, precond="vcycle", precision="f32_ir", inner_tol=itol, tol=1e-12)
        assert info["status"] == 0
        steps.append(info["ir_steps"])
    assert steps[0] >= steps[1]


def test_refinement_options(rr, case):
    name, P, R = case
    with pytest.raises(rr.RRError):
        R.solve(1.0, P.y, precision=7)
    with pytest.raises(rr.RRError):
        R.solve(1.0, P.y, precond="additive", precision="f32_ir")
    with pytest.raises(rr.RRError):
        R.solve(1.0, P.y, precision="f32_ir", krylov="fcg")
    with pytest.raises(rr.RRError):
        R.solve(1.0, P.y, precision="f32_ir", inner_tol=2.0)
    Q = datagen.sparse_problem(300, 80, 5, seed=1)
    Xv = Q.X.copy()
    Xv.data = np.random.default_rng(0).uniform(0.5, 2.0, Xv.nnz)
    Rv = rr.Ridge(Xv, n_clusters=0)
    with pytest.raises(rr.RRError):
        Rv.solve(1.0, Q.y, precond="jacobi", precision="f32_ir")


@pytest.mark.parametrize("lam", [1e-2, 1.0])
def test_fp32_cycle_keeps_the_fp64_krylov_space(rr, case, lam):
    """FP64 flexible CG whose V(1,1) cycle runs in FP32: one solve reaches
    the FP64 solution (no refinement restarts), in about the iterations of
    the all-FP64 flexible CG."""
    name, P, R = case
    wst = krylov.reference_solution(P.X, P.y, lam)
    w, info = R.solve(lam, P.y, precond="vcycle", krylov="fcg", fcg_m=1, precision="f32_cycle",
                      tol=1e-13, max_iter=20000)
    w64, i64 = R.solve(lam, P.y, precond="vcycle", krylov="fcg", fcg_m=1, tol=1e-13, max_iter=20000)
    err = np.linalg.norm(host(w) - wst) / np.linalg.norm(wst)
    err64 = np.linalg.norm(host(w64) - wst) / np.linalg.norm(wst)
    print(f"[mixed {name}] FP32 cycle lambda={lam}: {info['iters']} iterations (FP64 {i64['iters']}), "
          f"true residual {info['true_relres']:.1e}, error {err:.1e} (FP64 {err64:.1e})", flush=True)
    assert info["status"] == 0 and info["true_relres"] <= 1e-12
    assert err <= max(1e-10, 10 * err64)
    assert info["iters"] <= 1.25 * i64["iters"] + 2
    with pytest.raises(rr.RRError):   # the FP32 cycle needs flexible CG and V(1,1)
        R.solve(lam, P.y, precond="vcycle", precision="f32_cycle")
    with pytest.raises(rr.RRError):
        R.solve(lam, P.y, precond="jacobi", krylov="fcg", precision="f32_cycle")
