"""Autotuned sliced plans (rr_setup_opts.autotune): the tuner picks the
row pass's lanes per row among {1, 2, 4} (and 8, 16 for rows of 64 entries
or more on average) and the column pass's lane-stream divisor among
{1, 2, 4} by timing, caches it per device
and shape bucket, and the tuned plans compute the same operator (bit-exact
on integer vectors) and solve to the oracle's converged iterate."""
import numpy as np
import pytest

import datagen
from oracle import kmeans, krylov, operator as op

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


def test_autotune_choice_cache_and_results(rr):
    P = datagen.mid_sparse()
    print("[autotune] mid case", flush=True)
    R1 = rr.Ridge(P.X, n_clusters=100, seed=4, autotune=True)
    i1 = R1.info
    assert i1["tuned_rows_div"] in (1, 2, 4) and i1["tuned_cols_div"] in (1, 2, 4)
    R2 = rr.Ridge(P.X, n_clusters=100, seed=4, autotune=True)
    i2 = R2.info
    assert i2["tune_cached"] == 1
    assert (i2["tuned_rows_div"], i2["tuned_cols_div"]) == (i1["tuned_rows_div"], i1["tuned_cols_div"])
    v = np.random.default_rng(3).integers(-50, 50, P.X.shape[1]).astype(np.float64)
    got = host(R1.apply_operator(0.0, v))
    ref = op.apply_A(P.X, 0.0, v)
    assert np.array_equal(got, ref)
    lab, fc, it, centres = kmeans.kmeans_features(P.X, 100, 4)
    x_t, inf_t = krylov.solve(P.X, P.y, 1.0, "vcycle", lab, fc, tol=1e-13, max_iter=5000)
    w, info = R1.solve(1.0, P.y, precond="vcycle", fixed_iters=inf_t.iters)
    assert np.linalg.norm(host(w) - x_t) <= 1e-10 * np.linalg.norm(x_t)


def test_long_rows_lanes(rr):
    """Rows of about 300 entries: the default takes 8 lanes per row, the
    tuner chooses among 1 to 16; both plans give the exact operator on an
    integer vector, and the handle with the tuned plan solves to the
    oracle's converged iterate."""
    P = datagen.sparse_problem(3000, 6000, 300, seed=93)
    v = np.random.default_rng(4).integers(-50, 50, P.X.shape[1]).astype(np.float64)
    ref = op.apply_A(P.X, 0.0, v)
    R0 = rr.Ridge(P.X)
    assert R0.info["tuned_rows_div"] == 8
    assert np.array_equal(host(R0.apply_operator(0.0, v)), ref)
    R0.close()
    R = rr.Ridge(P.X, autotune=True)
    print(f"[autotune] long rows: {R.info['tuned_rows_div']} lanes per row", flush=True)
    assert R.info["tuned_rows_div"] in (1, 2, 4, 8, 16)
    assert np.array_equal(host(R.apply_operator(0.0, v)), ref)
    x, inf = krylov.solve(P.X, P.y, 2.0, "jacobi", tol=1e-13)
    w, info = R.solve(2.0, P.y, precond="jacobi", fixed_iters=inf.iters)
    assert np.linalg.norm(host(w) - x) <= 1e-10 * np.linalg.norm(x)
    R.close()
