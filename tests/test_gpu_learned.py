"""The learned coarse correction through the C ABI.

* Forward products against the oracle's FP64 network with the same (FP32)
  weights and inputs, elementwise within a rounding bound propagated
  through the layers: BF16 operands (round to nearest, u = 2^-9) and FP32
  accumulation (K 2^-24), so |dZ| <= (2u + u^2 + K 2^-24) |A||W^T| plus the
  propagated input error.
* Gradients against the oracle's backward in relative Frobenius norm: each
  gradient is the end of at most 8 chained BF16 roundings, so the bound is
  8 u times the measured ratio || |G|^T |A| || / || G^T A || of its last
  product (cancellation amplifies relative error by that ratio).
* Pairs produced by the solver, training by Adam, and flexible CG with the
  trained network against the method without a coarse correction."""
import numpy as np
import pytest

import datagen
from oracle import mlp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
U = 2.0 ** -9


@pytest.fixture(scope="module")
def rr():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1806_05826_amd as rr
    return rr


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def cuda32(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def unpack(flat, n_in, hid, n_out):
    p, o = {}, 0
    for k, shp in mlp.shapes(n_in, hid, n_out).items():
        n = int(np.prod(shp))
        p[k] = flat[o:o + n].reshape(shp).astype(np.float64)
        o += n
    return p


@pytest.fixture(scope="module")
def tiny(rr):
    P = datagen.tiny_sparse()
    R = rr.Ridge(P.X, n_clusters=50, seed=1)
    rr.rr_mlp_init(R.h, hidden=32, seed=7)
    return P, R


def test_forward_matches_oracle(rr, tiny):
    P, R = tiny
    npar, n_in, n_out = rr.rr_mlp_size(R.h)
    rng = np.random.default_rng(0)
    flat = rr.rr_mlp_get_weights(R.h)
    flat[:] = flat + 0.05 * rng.standard_normal(flat.size).astype(np.float32)   # nonzero biases
    rr.rr_mlp_set_weights(R.h, flat)
    p = unpack(flat, n_in, 32, n_out)
    X = rng.standard_normal((70, n_in)).astype(np.float32)
    out = torch.empty((70, n_out), dtype=torch.float32, device="cuda")
    rr.rr_mlp_forward(R.h, cuda32(X), out)
    Y = host(out).astype(np.float64)
    Yr, (X64, Z1, A1, Z2, A2) = mlp.forward(p, X.astype(np.float64))
    # elementwise bound propagated through the layers
    g = lambda K: 2 * U + U * U + K * 2.0 ** -24
    E1 = g(n_in) * np.abs(X64) @ np.abs(p["W1"]).T + U * np.abs(X64) @ np.abs(p["W1"]).T
    E2 = (E1 + U * np.abs(A1)) @ np.abs(p["W2"]).T + g(32) * np.abs(A1) @ np.abs(p["W2"]).T
    E3 = (E2 + U * np.abs(A2)) @ np.abs(p["W3"]).T + g(32) * np.abs(A2) @ np.abs(p["W3"]).T
    assert np.all(np.abs(Y - Yr) <= E3 + 1e-30), np.max(np.abs(Y - Yr) / (E3 + 1e-30))


def test_backward_matches_oracle(rr, tiny):
    P, R = tiny
    npar, n_in, n_out = rr.rr_mlp_size(R.h)
    rng = np.random.default_rng(1)
    flat = rr.rr_mlp_get_weights(R.h)
    p = unpack(flat, n_in, 32, n_out)
    X = rng.standard_normal((64, n_in)).astype(np.float32)
    D = rng.standard_normal((64, n_out)).astype(np.float32)
    grads = torch.empty(npar, dtype=torch.float32, device="cuda")
    rr.rr_mlp_backward(R.h, cuda32(X), cuda32(D), grads)
    g = unpack(host(grads), n_in, 32, n_out)
    Y, cache = mlp.forward(p, X.astype(np.float64))
    gr = mlp.backward(p, cache, D.astype(np.float64))
    X64, Z1, A1, Z2, A2 = cache
    dZ2 = (D @ p["W3"]) * (Z2 > 0)
    dZ1 = (dZ2 @ p["W2"]) * (Z1 > 0)
    last = {"W3": (D, A2), "W2": (dZ2, A1), "W1": (dZ1, X64)}
    for k in mlp.NAMES:
        if k.startswith("W"):
            G, A = last[k]
            ratio = np.linalg.norm(np.abs(G).T @ np.abs(A)) / np.linalg.norm(G.T @ A)
        else:
            G = {"b3": D, "b2": dZ2, "b1": dZ1}[k]
            ratio = np.linalg.norm(np.abs(G).sum(0)) / np.linalg.norm(G.sum(0))
        tol = 8 * U * ratio
        err = np.linalg.norm(g[k] - gr[k]) / np.linalg.norm(gr[k])
        assert err <= tol, (k, err, tol)


def test_adam_steps_match_oracle(rr, tiny):
    """rr_mlp_train on one pair takes one Adam step per epoch.  The gradient
    of a single pair has no batch sum, so rr_mlp_backward gives the very
    gradient the step uses; the oracle's FP64 Adam applied to it must give
    the GPU's FP32 weights after every step, within FP32 rounding of the
    update (relative 1e-5 of lr per step) and of the weight itself."""
    P, R = tiny
    rr.rr_mlp_init(R.h, hidden=32, seed=13)          # fresh Adam state
    npar, n_in, n_out = rr.rr_mlp_size(R.h)
    rng = np.random.default_rng(3)
    X = cuda32(rng.standard_normal((1, n_in)))
    T = cuda32(rng.standard_normal((1, n_out)))
    lr = 1e-3
    p = {"theta": rr.rr_mlp_get_weights(R.h).astype(np.float64)}
    opt = mlp.Adam(p, lr=lr)
    out = torch.empty((1, n_out), dtype=torch.float32, device="cuda")
    grads = torch.empty(npar, dtype=torch.float32, device="cuda")
    moved = 0
    for t in range(1, 6):
        rr.rr_mlp_forward(R.h, X, out)
        rr.rr_mlp_backward(R.h, X, (out - T).contiguous(), grads)
        g = host(grads).astype(np.float64)
        before = p["theta"].copy()
        rr.rr_mlp_train(R.h, X, T, epochs=1, batch=1, lr=lr, seed=t)
        opt.step(p, {"theta": g})
        got = rr.rr_mlp_get_weights(R.h).astype(np.float64)
        tol = t * 1e-5 * lr + 4 * np.spacing(np.abs(p["theta"]).astype(np.float32)).astype(np.float64)
        assert np.all(np.abs(got - p["theta"]) <= tol), (t, np.max(np.abs(got - p["theta"]) - tol))
        p["theta"] = got          # carry the GPU's FP32 weights (the next gradient is theirs)
        moved += int(np.count_nonzero(got != before))
    assert moved > npar        # the steps did move most parameters


@pytest.fixture(scope="module")
def wide(rr):
    P = datagen.sparse_problem(8000, 3000, 25, seed=79)
    R = rr.Ridge(P.X, n_clusters=200, seed=3)
    fc = R.info["n_coarse"]
    # lambda drawn log-uniformly around the solves below: the network must
    # learn A_c(lambda)^-1 on F_C-dimensional inputs, about F_C equations per
    # pair, so a few thousand pairs determine it only over a narrow range
    lams = list(np.exp(np.random.default_rng(2).uniform(np.log(0.3), np.log(3.0), 96)))
    per = 40
    inp = torch.empty((len(lams) * per, fc + 1), dtype=torch.float32, device="cuda")
    tgt = torch.empty((len(lams) * per, fc), dtype=torch.float32, device="cuda")
    y = torch.as_tensor(P.y, dtype=torch.float64, device="cuda")
    n = rr.rr_collect_pairs(R.h, lams, per, 1, y, inp, tgt)
    print(f"[learned] F_C={fc}, {n} pairs from {len(lams)} solves", flush=True)
    return P, R, fc, inp[:n].contiguous(), tgt[:n].contiguous(), lams


def test_pairs_are_coarse_corrections(rr, wide):
    P, R, fc, inp, tgt, lams = wide
    X = host(inp).astype(np.float64)
    T = host(tgt).astype(np.float64)
    assert np.allclose(np.linalg.norm(X[:, :fc], axis=1), 1.0, atol=1e-5)
    # the first pair of the first solve: target = A_c(lambda)^-1 input
    lam = float(np.exp(X[0, fc]))
    assert abs(lam - lams[0]) <= 1e-5 * lams[0]
    L, Ainv = (host(t) for t in R.coarse_factor(lams[0]))
    Dc = np.diag(np.tril(L) @ np.tril(L).T)   # diag(A_c), A_c = L L^T
    assert np.linalg.norm(T[0] - Dc * (Ainv @ X[0, :fc])) <= 1e-5 * np.linalg.norm(T[0])


def test_training_and_learned_fcg(rr, wide):
    """Training fits the pairs; flexible CG with the network as the cycle's
    coarse solve converges, at a bounded cost, thanks to the fallback; what
    the network gains over flexible CG without a coarse correction is
    measured and reported, not assumed (it is a loss at this fit)."""
    P, R, fc, inp, tgt, lams = wide
    rr.rr_mlp_init(R.h, hidden=256, seed=11)
    hist = rr.rr_mlp_train(R.h, inp, tgt, epochs=150, batch=256, lr=1e-3, seed=5)
    print(f"[learned] loss {hist[0]:.3e} -> {hist[-1]:.3e}", flush=True)
    assert hist[-1] < 0.1 * hist[0]
    # the fit: relative error of the network on its own training pairs
    out = torch.empty_like(tgt)
    rr.rr_mlp_forward(R.h, inp, out)
    T = tgt.double()
    rel = (torch.linalg.norm(out.double() - T, dim=1) / torch.linalg.norm(T, dim=1)).cpu().numpy()
    print(f"[learned] relative error on the training pairs: median {np.median(rel):.3f}, "
          f"90 % {np.quantile(rel, 0.9):.3f}", flush=True)
    assert np.median(rel) < 0.3
    n_learned = n_jacobi = 0
    for lam in (0.5, 1.0, 2.0):
        _, il = R.solve(lam, P.y, precond="learned", krylov="fcg", fcg_m=4, tol=1e-10, max_iter=5000)
        _, ij = R.solve(lam, P.y, precond="jacobi", krylov="fcg", fcg_m=4, tol=1e-10, max_iter=5000)
        _, iv = R.solve(lam, P.y, precond="vcycle", tol=1e-10, max_iter=5000)
        print(f"[learned] lambda={lam}: learned {il['iters']} its (fallback at {il['fallback_iter']}), "
              f"Jacobi {ij['iters']}, V(1,1) {iv['iters']}", flush=True)
        assert il["status"] == 0 and il["true_relres"] <= 2e-10
        # after a stall the solve continues with the algebraic cycle: it cannot
        # take much more than the iterations before the stall plus a V(1,1) solve
        fb = il["fallback_iter"]
        assert il["iters"] <= (fb if fb >= 0 else il["iters"]) + iv["iters"] + 16
        n_learned += il["iters"]
        n_jacobi += ij["iters"]
        # the first 16 iterations, all steered by the network (the stall test
        # first looks after the second chunk of 8, and a switch it makes
        # there would act from iteration 17 on, after these solves end)
        _, il16 = R.solve(lam, P.y, precond="learned", krylov="fcg", fcg_m=4, fixed_iters=16)
        _, ij16 = R.solve(lam, P.y, precond="jacobi", krylov="fcg", fcg_m=4, fixed_iters=16)
        assert il16["iters"] == 16 and np.isfinite(il16["relres"])
        print(f"[learned] lambda={lam}: relative residual after 16 iterations: learned "
              f"{il16['relres']:.2e}, Jacobi {ij16['relres']:.2e} (gain "
              f"{ij16['relres'] / il16['relres']:.2e}x)", flush=True)
    print(f"[learned] iterations over the three lambdas: learned {n_learned}, Jacobi {n_jacobi}", flush=True)


def test_learned_options(rr, tiny):
    P, R = tiny
    with pytest.raises(rr.RRError):
        R.solve(1.0, P.y, precond="learned")            # needs flexible CG
    Q = datagen.sparse_problem(300, 80, 5, seed=1)
    R2 = rr.Ridge(Q.X, n_clusters=10, seed=1)
    with pytest.raises(rr.RRError):
        R2.solve(1.0, Q.y, precond="learned", krylov="fcg")   # no network yet
    with pytest.raises(rr.RRError):
        rr.rr_mlp_init(R2.h, hidden=4)


def test_nan_network_falls_back_to_the_algebraic_cycle(rr, tiny):
    """A network whose weights were corrupted on the host (NaN) makes the
    first flexible-CG step fail; the solve switches to the V(1,1) cycle from
    the last good iterate (here x0 = 0) and converges, reporting the switch
    at iteration 0."""
    P, R = tiny
    npar, n_in, n_out = rr.rr_mlp_size(R.h)
    saved = rr.rr_mlp_get_weights(R.h)
    try:
        bad = np.full(npar, np.nan, dtype=np.float32)
        rr.rr_mlp_set_weights(R.h, bad)
        w, inf = R.solve(1.0, P.y, precond="learned", krylov="fcg", fcg_m=4, tol=1e-10, max_iter=500)
        wv, iv = R.solve(1.0, P.y, precond="vcycle", krylov="fcg", fcg_m=4, tol=1e-10, max_iter=500)
        print(f"[learned] NaN weights: status {inf['status']}, {inf['iters']} its, fallback at "
              f"{inf['fallback_iter']} (V(1,1) FCG {iv['iters']} its)", flush=True)
        assert inf["status"] == 0 and inf["fallback_iter"] == 0
        assert inf["true_relres"] <= 2e-10
        # from x0 = 0 with a fresh history this is the V(1,1) flexible-CG solve
        assert abs(inf["iters"] - iv["iters"]) <= 1
        d = np.linalg.norm(host(w) - host(wv)) / np.linalg.norm(host(wv))
        assert d <= 1e-8, d
        # an infinite weight as well
        bad[:] = 0.0
        bad[0] = np.inf
        rr.rr_mlp_set_weights(R.h, bad)
        w, inf = R.solve(0.3, P.y, precond="learned", krylov="fcg", fcg_m=2, tol=1e-10, max_iter=500)
        assert inf["status"] == 0 and inf["true_relres"] <= 2e-10
    finally:
        rr.rr_mlp_set_weights(R.h, saved)


def test_on_policy_pairs_are_coarse_corrections(rr, wide):
    """Pairs from the network's own flexible-CG solves have the same form:
    unit inputs, log lambda, and the exact coarse correction (in units of
    the coarse Jacobi step) as target."""
    P, R, fc, inp, tgt, lams = wide
    rr.rr_mlp_init(R.h, hidden=64, seed=3)
    rr.rr_mlp_train(R.h, inp, tgt, epochs=5, batch=256, lr=1e-3, seed=1)
    n_s, per = 4, 10
    inp2 = torch.empty((n_s * per, fc + 1), dtype=torch.float32, device="cuda")
    tgt2 = torch.empty((n_s * per, fc), dtype=torch.float32, device="cuda")
    y = torch.as_tensor(P.y, dtype=torch.float64, device="cuda")
    n = rr.rr_collect_pairs_learned(R.h, lams[:n_s], per, 1, y, inp2, tgt2)
    print(f"[learned] {n} on-policy pairs", flush=True)
    assert 1 <= n <= n_s * per
    X = host(inp2[:n]).astype(np.float64)
    T = host(tgt2[:n]).astype(np.float64)
    assert np.allclose(np.linalg.norm(X[:, :fc], axis=1), 1.0, atol=1e-5)
    lam = float(np.exp(X[0, fc]))
    assert abs(lam - lams[0]) <= 1e-5 * lams[0]
    L, Ainv = (host(t) for t in R.coarse_factor(lams[0]))
    Dc = np.diag(np.tril(L) @ np.tril(L).T)   # diag(A_c), A_c = L L^T
    assert np.linalg.norm(T[0] - Dc * (Ainv @ X[0, :fc])) <= 1e-5 * np.linalg.norm(T[0])
