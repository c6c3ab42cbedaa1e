"""The learned coarse-correction surrogate: a three-layer perceptron, FP64.

Test infrastructure (only tests/, __graft_entry__.smoke() and bench.py's CPU
baseline use it).  The network is not part of the paper; the paper's flexible
CG (its flexible-CG algorithm) is what lets a nonlinear preconditioner like
this one be used at all.

Network: in = F_C + 1 inputs [r_c / ||r_c||, log lambda] (r_c = P^T r),
two hidden layers of H units with ReLU, out = F_C outputs; the coarse
correction is c = ||r_c|| y.  Trained to reproduce the algebraic coarse
correction A_c(lambda)^-1 r_c / ||r_c|| under the loss
L = (1 / 2B) sum_b ||y_b - t_b||^2 with Adam.

Weights (row-major): W1 [H, in], b1 [H], W2 [H, H], b2 [H], W3 [out, H], b3 [out].
"""
from __future__ import annotations

import numpy as np

NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def shapes(n_in: int, hidden: int, n_out: int):
    return {"W1": (hidden, n_in), "b1": (hidden,), "W2": (hidden, hidden), "b2": (hidden,),
            "W3": (n_out, hidden), "b3": (n_out,)}


def init(n_in: int, hidden: int, n_out: int, rng) -> dict:
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases."""
    p = {}
    for name, shp in shapes(n_in, hidden, n_out).items():
        if name.startswith("W"):
            bound = np.sqrt(6.0 / shp[1])
            p[name] = rng.uniform(-bound, bound, shp)
        else:
            p[name] = np.zeros(shp)
    return p


def forward(p: dict, X: np.ndarray):
    """Returns the output Y [B, out] and the cache of pre-activations."""
    Z1 = X @ p["W1"].T + p["b1"]
    A1 = np.maximum(Z1, 0.0)
    Z2 = A1 @ p["W2"].T + p["b2"]
    A2 = np.maximum(Z2, 0.0)
    Y = A2 @ p["W3"].T + p["b3"]
    return Y, (X, Z1, A1, Z2, A2)


def loss(Y: np.ndarray, T: np.ndarray) -> float:
    return 0.5 * float(np.sum((Y - T) ** 2)) / Y.shape[0]


def backward(p: dict, cache, dY: np.ndarray) -> dict:
    """Gradients of a scalar whose derivative with respect to Y is dY."""
    X, Z1, A1, Z2, A2 = cache
    g = {}
    g["W3"] = dY.T @ A2
    g["b3"] = dY.sum(axis=0)
    dZ2 = (dY @ p["W3"]) * (Z2 > 0)
    g["W2"] = dZ2.T @ A1
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ p["W2"]) * (Z1 > 0)
    g["W1"] = dZ1.T @ X
    g["b1"] = dZ1.sum(axis=0)
    return g


def loss_grad(p: dict, X: np.ndarray, T: np.ndarray):
    Y, cache = forward(p, X)
    return loss(Y, T), backward(p, cache, (Y - T) / X.shape[0])


class Adam:
    """Kingma & Ba's Adam with bias correction: m = b1 m + (1-b1) g,
    v = b2 v + (1-b2) g^2, theta -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)."""

    def __init__(self, p: dict, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = {k: np.zeros_like(v) for k, v in p.items()}
        self.v = {k: np.zeros_like(v) for k, v in p.items()}
        self.t = 0

    def step(self, p: dict, g: dict):
        self.t += 1
        for k in p:
            self.m[k] = self.b1 * self.m[k] + (1 - self.b1) * g[k]
            self.v[k] = self.b2 * self.v[k] + (1 - self.b2) * g[k] ** 2
            mh = self.m[k] / (1 - self.b1 ** self.t)
            vh = self.v[k] / (1 - self.b2 ** self.t)
            p[k] = p[k] - self.lr * mh / (np.sqrt(vh) + self.eps)


def features(r_c: np.ndarray, lam: float):
    """Network input and scale for one coarse residual: ([r_c/||r_c||, log lam], ||r_c||)."""
    nrm = float(np.linalg.norm(r_c))
    x = np.concatenate([r_c / nrm if nrm > 0 else r_c, [np.log(lam)]])
    return x, nrm


def coarse_correction(p: dict, r_c: np.ndarray, lam: float) -> np.ndarray:
    x, nrm = features(r_c, lam)
    y, _ = forward(p, x[None, :])
    return nrm * y[0]
