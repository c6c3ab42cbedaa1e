"""Pins of the oracle's learned coarse correction (oracle/mlp.py)."""
import numpy as np
import pytest

from oracle import mlp


def small(seed=0, n_in=7, hidden=5, n_out=4, B=6):
    rng = np.random.default_rng(seed)
    p = mlp.init(n_in, hidden, n_out, rng)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.standard_normal(p[k].shape) * 0.1
    X = rng.standard_normal((B, n_in))
    T = rng.standard_normal((B, n_out))
    return p, X, T


def test_gradients_match_central_differences():
    p, X, T = small()
    L, g = mlp.loss_grad(p, X, T)
    h = 1e-6
    for k in mlp.NAMES:
        num = np.zeros_like(p[k])
        it = np.nditer(p[k], flags=["multi_index"])
        for _ in it:
            i = it.multi_index
            old = p[k][i]
            p[k][i] = old + h
            Lp = mlp.loss(mlp.forward(p, X)[0], T)
            p[k][i] = old - h
            Lm = mlp.loss(mlp.forward(p, X)[0], T)
            p[k][i] = old
            num[i] = (Lp - Lm) / (2 * h)
        assert np.max(np.abs(num - g[k])) <= 1e-7 * max(1.0, np.max(np.abs(g[k]))), k


def test_linear_regime_closed_form():
    # with all pre-activations positive the network is affine; the output
    # gradient of the loss is then (Y - T)/B pushed through W3 W2 exactly
    p, X, T = small(seed=3)
    p["W2"] = np.abs(p["W2"])
    for k in ("b1", "b2"):
        p[k] = p[k] + 100.0   # every unit active
    Z1 = X @ p["W1"].T + p["b1"]
    assert np.all(Z1 > 0) and np.all(Z1 @ p["W2"].T + p["b2"] > 0)
    Y, cache = mlp.forward(p, X)
    A = p["W3"] @ p["W2"] @ p["W1"]
    c = p["W3"] @ (p["W2"] @ p["b1"] + p["b2"]) + p["b3"]
    assert np.allclose(Y, X @ A.T + c, rtol=0, atol=1e-10)
    g = mlp.backward(p, cache, (Y - T) / X.shape[0])
    G = (Y - T) / X.shape[0]
    assert np.allclose(g["W1"], (G @ p["W3"] @ p["W2"]).T @ X, atol=1e-12)
    assert np.allclose(g["b3"], G.sum(axis=0), atol=1e-15)


def test_adam_first_step_is_sign_step():
    # after one step the bias-corrected moments are g and g^2, so every
    # parameter moves by lr * g / (|g| + eps)
    p, X, T = small(seed=4)
    q = {k: v.copy() for k, v in p.items()}
    _, g = mlp.loss_grad(p, X, T)
    opt = mlp.Adam(p, lr=0.01)
    opt.step(p, g)
    for k in p:
        assert np.allclose(q[k] - p[k], 0.01 * g[k] / (np.abs(g[k]) + 1e-8), rtol=1e-12, atol=0)


def test_training_fits_a_linear_map():
    # the map the network learns in the solver, r_c -> A^-1 r_c / ||r_c||, is
    # linear in the normalized input: Adam on it reduces the loss by orders
    rng = np.random.default_rng(5)
    n = 6
    M = rng.standard_normal((n, n))
    A = M @ M.T + n * np.eye(n)
    R = rng.standard_normal((400, n))
    R /= np.linalg.norm(R, axis=1, keepdims=True)
    X = np.hstack([R, np.zeros((400, 1))])
    T = np.linalg.solve(A, R.T).T
    p = mlp.init(n + 1, 32, n, rng)
    opt = mlp.Adam(p, lr=3e-3)
    L0 = mlp.loss(mlp.forward(p, X)[0], T)
    for _ in range(1500):
        L, g = mlp.loss_grad(p, X, T)
        opt.step(p, g)
    assert L < 1e-3 * L0


def test_features_and_scale_invariance():
    rng = np.random.default_rng(6)
    p = mlp.init(5, 8, 4, rng)
    r = rng.standard_normal(4)
    c1 = mlp.coarse_correction(p, r, 0.5)
    c2 = mlp.coarse_correction(p, 3.0 * r, 0.5)
    assert np.allclose(c2, 3.0 * c1, rtol=1e-13)
    x, nrm = mlp.features(r, 0.5)
    assert x[-1] == np.log(0.5) and abs(np.linalg.norm(x[:-1]) - 1) < 1e-15


def test_adam_constant_gradient_closed_form():
    """With the same gradient g at every step the bias-corrected moments are
    exactly g and g^2, so after t steps theta = theta0 - t lr g / (|g| + eps);
    a missing or shifted bias correction breaks this from the second step."""
    rng = np.random.default_rng(21)
    p = {"W": rng.standard_normal((3, 4)), "b": rng.standard_normal(3)}
    g = {"W": rng.standard_normal((3, 4)), "b": np.array([2e-8, -3.0, 0.5])}
    theta0 = {k: v.copy() for k, v in p.items()}
    opt = mlp.Adam(p, lr=1e-2, eps=1e-8)
    for t in range(1, 8):
        opt.step(p, g)
        for k in p:
            ref = theta0[k] - t * 1e-2 * g[k] / (np.abs(g[k]) + 1e-8)
            assert np.allclose(p[k], ref, rtol=0, atol=1e-12 * t), (k, t)
