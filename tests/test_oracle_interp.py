"""Pins of the least-squares interpolation oracle (the paper's least-squares
interpolation subsection) against brute force, exact interpolation of one
prototype, the Galerkin projection property and the adjusted square-root
average it reduces to."""
import numpy as np
import pytest
import scipy.optimize as so
import scipy.sparse as sp

import datagen
from oracle import interp, leader, precond
from oracle.operator import apply_A


def _case(seed=0, F=40, K=3, fc=6):
    rng = np.random.default_rng(seed)
    labels = np.concatenate([np.arange(fc), rng.integers(0, fc, F - fc)])
    rng.shuffle(labels)
    V = rng.standard_normal((F, K))
    eta = rng.uniform(0.5, 4.0, K)
    return labels, fc, V, eta


def test_weights_minimise_the_weighted_error():
    labels, fc, V, eta = _case()
    rep = interp.representatives(labels, fc)
    p = interp.ls_weights(V, eta, labels, fc, rep)
    for i in range(len(labels)):
        r = rep[labels[i]]
        res = so.minimize_scalar(lambda t: float(np.sum(eta * (V[i] - t * V[r]) ** 2)),
                                 method="brent", options={"xtol": 1e-13})
        assert abs(p[i] - res.x) <= 1e-7 * max(1.0, abs(res.x)), (i, p[i], res.x)
    # the representative interpolates itself exactly
    assert np.allclose(p[rep], 1.0, rtol=4e-16, atol=0)


def test_representatives_are_lowest_members_and_lf_leaders():
    labels = np.array([2, 0, 2, 1, 0, 1, 2])
    assert list(interp.representatives(labels, 3)) == [1, 3, 0]
    with pytest.raises(ValueError):
        interp.representatives(np.array([0, 0, 2]), 3)
    X = datagen.zipf_binary_csr(300, 120, 6, 1.1, 5)
    lab, fc, leaders = leader.leader_follower(X, 3.0)
    assert np.array_equal(interp.representatives(lab, fc), leaders)


def test_one_prototype_is_interpolated_exactly():
    labels, fc, V, eta = _case(1, K=1)
    rep = interp.representatives(labels, fc)
    p = interp.ls_weights(V, eta, labels, fc, rep)
    P = interp.ls_prolongation(labels, fc, p)
    v = V[:, 0]
    assert np.allclose(P @ v[rep], v, rtol=1e-14, atol=1e-15)


def test_cluster_constant_prototypes_give_plain_aggregation():
    rng = np.random.default_rng(2)
    labels, fc, _, eta = _case(2)
    W = rng.standard_normal((fc, 3))
    V = W[labels]                     # constant within every cluster
    p = interp.ls_weights(V, eta, labels, fc, interp.representatives(labels, fc))
    assert np.allclose(p, 1.0, rtol=1e-14)


def test_zero_energy_representative_falls_back_to_aggregation():
    labels, fc, V, eta = _case(3)
    rep = interp.representatives(labels, fc)
    V[rep[2], :] = 0.0
    p = interp.ls_weights(V, eta, labels, fc, rep)
    assert np.all(p[labels == 2] == 1.0)
    assert not np.all(p[labels == 1] == 1.0)


def test_energies_are_the_operator_norms():
    X = datagen.zipf_binary_csr(200, 50, 5, 1.1, 7)
    rng = np.random.default_rng(4)
    V = rng.standard_normal((50, 4))
    beta = 0.7
    eta = interp.prototype_energies(X, V, beta)
    Xd = X.toarray()
    ref = np.sum((Xd @ V) ** 2, axis=0) + beta * np.sum(V ** 2, axis=0)
    assert np.allclose(eta, ref, rtol=1e-13)


def _ls_setup(seed=5, lam=0.5):
    X = datagen.zipf_binary_csr(400, 90, 6, 1.1, seed)
    lab, fc, _ = leader.leader_follower(X, 3.0)
    G = (X.T @ X).toarray()
    ev, Q = np.linalg.eigh(G)
    V = Q[:, ::-1][:, :4]             # the four principal components
    eta = interp.prototype_energies(X, V, lam)
    p = interp.ls_weights(V, eta, lab, fc, interp.representatives(lab, fc))
    return X, lab, fc, interp.ls_prolongation(lab, fc, p), lam


def test_galerkin_coarse_correction_is_exact_on_the_range_of_P():
    X, lab, fc, P, lam = _ls_setup()
    assert not np.allclose((P.T @ P).toarray(), np.eye(fc))
    tl = precond.TwoLevel(X, lam, lab, fc, 0.5, P=P)
    y = np.random.default_rng(6).standard_normal(fc)
    r = apply_A(X, lam, P @ y)
    assert np.allclose(tl.coarse_correction(r), P @ y, rtol=1e-9, atol=1e-11)
    # the coarse matrix is the Galerkin product with the dense A
    A = (X.T @ X).toarray() + lam * np.eye(X.shape[1])
    Pd = P.toarray()
    assert np.allclose(tl.Ac, Pd.T @ A @ Pd, rtol=1e-12, atol=1e-12)


def test_plain_aggregation_matches_the_square_root_average():
    X = datagen.zipf_binary_csr(300, 80, 6, 1.1, 8)
    lab, fc, _ = leader.leader_follower(X, 3.0)
    lam = 1.0
    P1 = interp.ls_prolongation(lab, fc, np.ones(80))
    a = precond.TwoLevel(X, lam, lab, fc, 0.5, P=P1)
    b = precond.TwoLevel(X, lam, lab, fc, 0.5)
    r = np.random.default_rng(9).standard_normal(80)
    assert np.allclose(a.coarse_correction(r), b.coarse_correction(r), rtol=1e-11, atol=1e-13)
    assert np.allclose(a.vcycle(r), b.vcycle(r), rtol=1e-11, atol=1e-13)


def test_leading_prototypes_closed_form_and_eigen_equation():
    """Disjoint column supports make X^T X diagonal with the squared column
    norms on it, so the leading prototypes are the unit vectors of the
    largest columns; on a general matrix every prototype satisfies
    X^T X v = mu v with mu the largest eigenvalues (checked against the
    singular values of X)."""
    # columns with disjoint supports and norms^2 = 1, 9, 4, 16 (integer rows)
    X = sp.csr_matrix(np.array([[1, 0, 0, 0], [0, 3, 0, 0], [0, 0, 2, 0], [0, 0, 0, 4.0]]))
    V, ev = interp.leading_prototypes(X, 2)
    assert np.allclose(ev, [16.0, 9.0])
    assert np.allclose(np.abs(V[:, 0]), [0, 0, 0, 1]) and np.allclose(np.abs(V[:, 1]), [0, 1, 0, 0])
    rng = np.random.default_rng(3)
    Y = sp.random(60, 25, density=0.2, random_state=rng, format="csr")
    V, ev = interp.leading_prototypes(Y, 5)
    sv = np.linalg.svd(Y.toarray(), compute_uv=False)
    assert np.allclose(ev, sv[:5] ** 2, rtol=1e-12)
    G = (Y.T @ Y).toarray()
    for k in range(5):
        assert np.linalg.norm(G @ V[:, k] - ev[k] * V[:, k]) <= 1e-12 * ev[0]
        assert abs(np.linalg.norm(V[:, k]) - 1.0) <= 1e-14
