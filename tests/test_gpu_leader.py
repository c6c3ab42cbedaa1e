"""GPU parity of leader-follower clustering (rr_setup_opts.lf_tolerance)
against the CPU oracle: labels and leaders bit-exact (exact integer
distances on both sides), and a two-level solve on that aggregation."""
import numpy as np
import pytest

import datagen
from oracle import krylov, leader

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
    "tiny": lambda: datagen.tiny_sparse().X,
    "ragged": lambda: datagen.sparse_problem(3001, 1237, 7, seed=77).X,
    "mid": lambda: datagen.mid_sparse().X,
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("tol", [2.5, 4.0])
def test_leader_follower_bit_exact(rr, name, tol):
    X = CASES[name]()
    lab, fc, lead = leader.leader_follower(X, tol)
    print(f"[lf {name} tol={tol}] F={X.shape[1]} F_C={fc}", flush=True)
    R = rr.Ridge(X, lf_tolerance=tol)
    assert R.info["n_coarse"] == fc
    assert np.array_equal(host(R.labels()), lab)
    assert np.array_equal(host(R.centres())[:fc], lead)
    R.close()


def test_leader_follower_duplicated_columns(rr):
    X, groups = datagen.duplicated_columns(400, [3, 1, 5, 2, 4], 0.05, seed=6)
    R = rr.Ridge(X, lf_tolerance=0.5)
    lab = host(R.labels())
    assert R.info["n_coarse"] == 5
    for g in range(5):
        assert len(set(lab[groups == g].tolist())) == 1


def test_leader_follower_solve(rr):
    P = datagen.mid_sparse()
    lab, fc, lead = leader.leader_follower(P.X, 4.0)
    R = rr.Ridge(P.X, lf_tolerance=4.0)
    x_t, inf = krylov.solve(P.X, P.y, 0.5, "vcycle", lab, fc, tol=1e-12)
    w, info = R.solve(0.5, P.y, precond="vcycle", fixed_iters=inf.iters)
    assert np.linalg.norm(host(w) - x_t) <= 1e-10 * np.linalg.norm(x_t)
