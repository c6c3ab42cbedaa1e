"""Batched solves (rr_solve_batched) through the C ABI.

Bars: every problem of a batch gives bitwise the result of its own rr_solve
(the kernels are deterministic, so running problems concurrently on their
handles' streams must not change a bit); uneven independent problems each
match the oracle's solution of their own system."""
import numpy as np
import pytest

import datagen
from oracle import kmeans, krylov

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


@pytest.fixture(scope="module")
def handles(rr):
    probs = [datagen.tiny_sparse(), datagen.sparse_problem(3001, 1237, 7, seed=77),
             datagen.sparse_problem(5000, 2000, 12, seed=78)]
    Rs = [rr.Ridge(P.X, n_clusters=k, seed=s) for P, k, s in zip(probs, (50, 80, 100), (1, 2, 3))]
    return probs, Rs


@pytest.mark.parametrize("krylov_kind", ["pcg", "fcg"])
def test_batch_equals_single_solves(rr, handles, krylov_kind):
    probs, Rs = handles
    # distinct handles run together; the first handle appears twice
    order = [0, 1, 2, 0]
    lams = [1.0, 0.3, 5.0, 0.01]
    rhs = [dev(probs[i].y) for i in order]
    ws = [torch.empty(probs[i].X.shape[1], dtype=torch.float64, device="cuda") for i in order]
    print(f"[batched] {krylov_kind} order {order}", flush=True)
    st, infos = rr.rr_solve_batched([Rs[i].h for i in order], lams, rhs, ws, tol=1e-10,
                                    precond="vcycle", krylov=krylov_kind)
    assert st == 0
    for j, i in enumerate(order):
        w1, inf1 = Rs[i].solve(lams[j], probs[i].y, precond="vcycle", tol=1e-10, krylov=krylov_kind)
        assert infos[j]["status"] == 0
        assert infos[j]["iters"] == inf1["iters"]
        assert np.array_equal(host(ws[j]), host(w1)), (j, i)
        assert infos[j]["true_relres"] == inf1["true_relres"]


def test_many_lambdas_on_one_handle(rr, handles):
    """Ten lambdas of one matrix: eight work sets in the first wave, two in
    the second, each result bitwise its single solve."""
    probs, Rs = handles
    P, R = probs[1], Rs[1]
    lams = list(np.logspace(-2, 2, 10))
    y = dev(P.y)
    ws = [torch.empty(P.X.shape[1], dtype=torch.float64, device="cuda") for _ in lams]
    print("[batched] 10 lambdas on one handle", flush=True)
    st, infos = rr.rr_solve_batched([R.h] * len(lams), lams, [y] * len(lams), ws, tol=1e-10,
                                    precond="vcycle")
    assert st == 0
    for lam, w, inf in zip(lams, ws, infos):
        w1, inf1 = R.solve(lam, P.y, precond="vcycle", tol=1e-10)
        assert inf["iters"] == inf1["iters"] and np.array_equal(host(w), host(w1))


def test_uneven_problems_match_oracle(rr):
    batch = datagen.batched_problems(6, seed=4, n_range=(500, 4000), d_range=(200, 1500))
    Rs, rhs, ws, lams = [], [], [], []
    for P, lam in batch:
        k = max(2, P.X.shape[1] // 10)
        Rs.append(rr.Ridge(P.X, n_clusters=k, seed=9))
        rhs.append(dev(P.y))
        ws.append(torch.empty(P.X.shape[1], dtype=torch.float64, device="cuda"))
        lams.append(lam)
    print(f"[batched] uneven sizes {[P.X.shape for P, _ in batch]}", flush=True)
    st, infos = rr.rr_solve_batched([R.h for R in Rs], lams, rhs, ws, tol=1e-12, max_iter=5000,
                                    precond="vcycle")
    assert st == 0
    for (P, lam), w, inf in zip(batch, ws, infos):
        wst = krylov.reference_solution(P.X, P.y, lam)
        assert inf["status"] == 0 and inf["relres"] <= 1e-12
        # error bounded by the residual through the condition number
        G = (P.X.T @ P.X).toarray() + lam * np.eye(P.X.shape[1])
        kappa = np.linalg.cond(G)
        err = np.linalg.norm(host(w) - wst) / np.linalg.norm(wst)
        assert err <= 2 * kappa * 1e-12 + 1e-13, (err, kappa)
    for (P, lam), R, w, inf in zip(batch, Rs, ws, infos):
        w1, inf1 = R.solve(lam, P.y, precond="vcycle", tol=1e-12, max_iter=5000)
        assert inf1["iters"] == inf["iters"] and np.array_equal(host(w1), host(w))


def test_batch_errors_and_empty(rr, handles):
    probs, Rs = handles
    st, infos = rr.rr_solve_batched([], [], [], [])
    assert st == 0 and infos == []
    y = dev(probs[0].y)
    w = torch.empty(probs[0].X.shape[1], dtype=torch.float64, device="cuda")
    # a bad lambda fails its own problem; the others still run
    y1 = dev(probs[1].y)
    w1 = torch.empty(probs[1].X.shape[1], dtype=torch.float64, device="cuda")
    st, infos = rr.rr_solve_batched([Rs[0].h, Rs[1].h], [-1.0, 1.0], [y, y1], [w, w1],
                                    precond="vcycle", raise_on=())
    assert st == 1 and infos[0]["status"] == 1 and infos[1]["status"] == 0
    w2, inf2 = Rs[1].solve(1.0, probs[1].y, precond="vcycle")
    assert np.array_equal(host(w1), host(w2))
