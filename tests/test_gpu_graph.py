"""PCG chunks captured in a HIP graph and replayed (rr_solve_opts.graph):
every replayed solve must give bitwise the eager solve's result, with eager
work and synchronizations between the replays, across lambdas (a new
signature re-captures), residual histories and fixed iteration counts."""
import numpy as np
import pytest

import datagen

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


@pytest.mark.parametrize("kind", ["vcycle", "additive", "jacobi", "none"])
def test_graph_replays_equal_eager(rr, kind):
    P = datagen.sparse_problem(3001, 1237, 7, seed=77)
    R = rr.Ridge(P.X, n_clusters=80, seed=2)
    print(f"[graph] {kind}", flush=True)
    for rep in range(3):
        for lam in (0.1, 1.0, 10.0):
            we, ie = R.solve(lam, P.y, precond=kind, tol=1e-10, chunk=4)
            wg, ig = R.solve(lam, P.y, precond=kind, tol=1e-10, chunk=4, graph=True)
            assert ie["iters"] == ig["iters"] and ie["status"] == ig["status"] == 0
            assert np.array_equal(host(we), host(wg)), (rep, lam)
            # eager work between replays on the same handle
            R.apply_operator(lam, np.ones(P.X.shape[1]))
    hist_e = torch.zeros(400, dtype=torch.float64, device="cuda")
    hist_g = torch.zeros(400, dtype=torch.float64, device="cuda")
    we, ie = R.solve(1.0, P.y, precond=kind, fixed_iters=21, residual_history=hist_e, chunk=4)
    wg, ig = R.solve(1.0, P.y, precond=kind, fixed_iters=21, residual_history=hist_g, chunk=4,
                     graph=True)
    assert ig["iters"] == 21 and np.array_equal(host(we), host(wg))
    assert np.array_equal(host(hist_e), host(hist_g))


def test_graph_on_a_side_stream(rr):
    P = datagen.tiny_sparse()
    R = rr.Ridge(P.X, n_clusters=50, seed=1)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        wg, ig = R.solve(1.0, P.y, precond="vcycle", tol=1e-10, graph=True)
    st.synchronize()
    we, ie = R.solve(1.0, P.y, precond="vcycle", tol=1e-10)
    assert np.array_equal(host(we), host(wg))
