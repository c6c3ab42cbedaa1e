"""Device memory through the C ABI: handles living in a caller workspace
(rr_setup_workspace_size / rr_setup_ws), PyTorch's caching allocator as the
library's allocator, and solves that allocate nothing once setup reserved
their buffers."""
import gc

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


def device_csr(X):
    X = X.tocsr()
    X.sort_indices()
    rp = torch.as_tensor(X.indptr.astype(np.int32), device="cuda")
    ci = torch.as_tensor(X.indices.astype(np.int32), device="cuda")
    return rp, ci


def test_workspace_handle_equals_allocated_handle(rr):
    P = datagen.sparse_problem(3001, 1237, 7, seed=77)
    rp, ci = device_csr(P.X)
    opts = dict(n_clusters=80, seed=2, reserve_fcg_m=2, reserve_f32=True)
    need = rr.rr_setup_workspace_size(rp, ci, None, P.X.shape[1], **opts)
    print(f"[memory] workspace of the 3001 x 1237 handle: {need} bytes", flush=True)
    assert need > 0
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    h_ws = rr.rr_setup_ws(rp, ci, None, P.X.shape[1], ws, **opts)
    h = rr.rr_setup(rp, ci, None, P.X.shape[1], **opts)
    y = torch.as_tensor(P.y, dtype=torch.float64, device="cuda")
    for kw in (dict(precond="vcycle"), dict(precond="vcycle", krylov="fcg", fcg_m=2),
               dict(precond="vcycle", precision="f32_ir")):
        w1 = torch.empty(P.X.shape[1], dtype=torch.float64, device="cuda")
        w2 = torch.empty_like(w1)
        st1, i1 = rr.rr_solve(h_ws, 0.7, y, w1, tol=1e-10, **kw)
        st2, i2 = rr.rr_solve(h, 0.7, y, w2, tol=1e-10, **kw)
        assert st1 == st2 == 0 and i1["iters"] == i2["iters"], kw
        assert np.array_equal(host(w1), host(w2)), kw
    # more flexible-CG directions than reserved: the workspace has no room
    w1 = torch.empty(P.X.shape[1], dtype=torch.float64, device="cuda")
    st, _ = rr.rr_solve(h_ws, 0.7, y, w1, krylov="fcg", fcg_m=8, raise_on=())
    assert st == rr.RR_ERR_WORKSPACE
    rr.rr_destroy(h_ws)
    rr.rr_destroy(h)
    # one byte short: setup fails cleanly
    small = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(rr.RRError) as e:
        rr.rr_setup_ws(rp, ci, None, P.X.shape[1], small, **opts)
    assert e.value.status == rr.RR_ERR_WORKSPACE
    del ws, small


def test_solves_allocate_nothing_after_reservation(rr):
    """With the flexible-CG ring, the refinement vectors and two extra work
    sets reserved at setup, the first solve of each kind leaves PyTorch's
    allocated bytes (every library allocation goes through its caching
    allocator) unchanged."""
    P = datagen.sparse_problem(5000, 2000, 12, seed=78)
    R = rr.Ridge(P.X, n_clusters=100, seed=3, lambda_slots=6, reserve_fcg_m=4, reserve_sets=2,
                 reserve_f32=True)
    y = torch.as_tensor(P.y, dtype=torch.float64, device="cuda")
    w = torch.empty(P.X.shape[1], dtype=torch.float64, device="cuda")
    ws = [torch.empty_like(w) for _ in range(3)]
    v = torch.randn(P.X.shape[1], dtype=torch.float64, device="cuda")
    out = torch.empty_like(v)
    gc.collect()   # objects of earlier tests must not be freed inside the measurements
    gc.disable()
    torch.cuda.synchronize()
    kinds = [
        ("vcycle", lambda: rr.rr_solve(R.h, 0.5, y, w, precond="vcycle")),
        ("additive", lambda: rr.rr_solve(R.h, 0.6, y, w, precond="additive", max_iter=3000)),
        ("jacobi", lambda: rr.rr_solve(R.h, 0.7, y, w, precond="jacobi", max_iter=3000)),
        ("fcg4", lambda: rr.rr_solve(R.h, 0.8, y, w, precond="vcycle", krylov="fcg", fcg_m=4)),
        ("f32_ir", lambda: rr.rr_solve(R.h, 0.9, y, w, precond="vcycle", precision="f32_ir")),
        ("batched", lambda: rr.rr_solve_batched([R.h] * 3, [1.1, 1.2, 1.3], [y] * 3, ws,
                                                precond="vcycle")),
        ("operator", lambda: rr.rr_apply_operator(R.h, 2.0, v, out)),
        ("precond", lambda: rr.rr_apply_precond(R.h, 0.5, "vcycle", 0.0, v, out)),
    ]
    try:
        for name, f in kinds:
            before = torch.cuda.memory_allocated()
            st = f()
            torch.cuda.synchronize()
            after = torch.cuda.memory_allocated()
            print(f"[memory] {name}: allocated {before} -> {after}", flush=True)
            assert (st[0] if isinstance(st, tuple) else 0) == 0, name
            assert after == before, name
    finally:
        gc.enable()
    R.close()


def test_library_memory_comes_from_torch(rr):
    """A handle's setup takes its device memory from PyTorch's caching
    allocator; destroying it gives the memory back."""
    P = datagen.tiny_sparse()
    gc.collect()   # objects of earlier tests must not be freed inside the measurement
    gc.disable()
    try:
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        R = rr.Ridge(P.X, n_clusters=50, seed=1)
        mid = torch.cuda.memory_allocated()
        R.close()
        torch.cuda.synchronize()
        after = torch.cuda.memory_allocated()
    finally:
        gc.enable()
    print(f"[memory] torch allocated: {before} -> {mid} -> {after}", flush=True)
    assert mid > before
    assert after == before
