"""The allocation-free persistent batched solve (rr_solve_batched_noalloc)
through the C ABI, against rr_solve_batched with persistent = 1: the same
kernel and the same problem order, so every result is bitwise equal.  Two
calls in a row, the second with fewer problems (the static scratch keeps the
first call's contents); the solve allocates nothing (PyTorch's allocated
bytes, which include all of the library's memory, do not move)."""
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


def test_noalloc_matches_persistent(rr):
    batch = datagen.batched_problems(9, seed=31, n_range=(500, 3000), d_range=(200, 1200))
    Rs = []
    for P, _ in batch:
        k = int(min(800, max(8, -(-P.X.shape[1] // 10))))
        Rs.append(rr.Ridge(P.X, n_clusters=k, seed=9, reserve_sets=1))
    # the first handle twice (a reserved work set), at another lambda
    order = list(range(len(batch))) + [0]
    lams = [lam for _, lam in batch] + [2.5]
    for n in (len(order), 4):   # the second call is smaller
        idx = order[:n]
        rhs = [torch.as_tensor(batch[i][0].y, dtype=torch.float64, device="cuda") for i in idx]
        w_ref = [torch.empty(batch[i][0].X.shape[1], dtype=torch.float64, device="cuda") for i in idx]
        w_new = [torch.empty_like(w) for w in w_ref]
        print(f"[noalloc] {n} problems", flush=True)
        st, inf_ref = rr.rr_solve_batched([Rs[i].h for i in idx], lams[:n], rhs, w_ref, tol=1e-10,
                                          precond="vcycle", persistent=True)
        assert st == 0
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        st, inf_new = rr.rr_solve_batched_noalloc([Rs[i].h for i in idx], lams[:n], rhs, w_new,
                                                  tol=1e-10, precond="vcycle")
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        assert st == 0
        for j in range(n):
            assert inf_new[j]["status"] == 0 and inf_new[j]["iters"] == inf_ref[j]["iters"], j
            assert inf_new[j]["true_relres"] == inf_ref[j]["true_relres"], j
            assert np.array_equal(host(w_new[j]), host(w_ref[j])), j


def test_noalloc_limits(rr):
    P = datagen.tiny_sparse()
    R = rr.Ridge(P.X, n_clusters=50, seed=1, lambda_slots=2)
    y = torch.as_tensor(P.y, dtype=torch.float64, device="cuda")
    ws = [torch.empty(P.X.shape[1], dtype=torch.float64, device="cuda") for _ in range(2)]
    # the handle twice without a reserved work set
    st, _ = rr.rr_solve_batched_noalloc([R.h, R.h], [1.0, 2.0], [y, y], ws, raise_on=())
    assert st == rr.RR_ERR_WORKSPACE
    # more problems than the scratch holds (rejected before any device work)
    many = 2049
    st, _ = rr.rr_solve_batched_noalloc([R.h] * many, [1.0] * many, [y] * many, [ws[0]] * many,
                                        raise_on=())
    assert st == rr.RR_ERR_INVALID_ARG
    R.close()
