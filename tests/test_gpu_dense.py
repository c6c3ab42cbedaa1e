"""GPU parity of the dense-X path (rr_setup_dense / rr_solve_block /
rr_apply_operator_block) against the CPU oracle on seeded block-correlated
Gaussian features (datagen.block_correlated_dense), sizes with ragged tails
against the 128-row and 128-column padding of the matrix-core tiles.

Bars: FP64 operator within a rigorous summation bound of the oracle's; the
BF16-operand operator within oracle.operator.apply_A_bf16_bound of its
definition; K = P^T X^T X P to 1e-12 of max|K|; FP64 block solves: natural
stops within the oracle's own spread under rounding-level changes +-1,
converged iterates within 1e-10 per column; the
BF16 refinement reaches the dense Cholesky solution to 1e-10."""
import numpy as np
import pytest

import datagen
from oracle import coarse, kmeans, krylov, operator as op, precond

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


@pytest.fixture(scope="module")
def small(rr):
    """1037 x 261, 37 blocks of 7 columns with correlation 0.9 inside a block
    (plus 2 free columns): every GEMM dimension has a ragged tile."""
    X = datagen.block_correlated_dense(1037, 37, 7, 0.9, seed=31)
    X = np.concatenate([X, datagen.block_correlated_dense(1037, 2, 1, 0.0, seed=32)], axis=1)
    print(f"[dense small] X {X.shape}", flush=True)
    return X.astype(np.float32)


def test_operator_f64_and_bf16(rr, small):
    X = small.astype(np.float64)
    R = rr.DenseRidge(small)
    assert R.info["dense"] == 1 and R.info["nnz"] == X.size
    rng = np.random.default_rng(5)
    for m in (1, 37, 130):
        V = rng.standard_normal((m, X.shape[1]))
        Q = host(R.apply_operator_block(0.7, V))
        for c in range(m):
            want = op.apply_A(X, 0.7, V[c])
            bound = 4 * (X.shape[0] + X.shape[1]) * 2.0**-53 * (np.abs(X).T @ (np.abs(X) @ np.abs(V[c])) + 0.7 * np.abs(V[c]))
            assert np.all(np.abs(Q[c] - want) <= bound), (m, c)
        Qb = host(R.apply_operator_block(0.7, V, precision="bf16_ir"))
        want_b = op.apply_A_bf16(X, 0.7, V.T).T
        bound_b = op.apply_A_bf16_bound(X, V.T).T + 1e-12 * np.abs(want_b)
        assert np.all(np.abs(Qb - want_b) <= bound_b), m
        # almost every U entry rounds the same way as the exact one
        rel = np.abs(Qb - want_b) / np.abs(want_b).max()
        assert np.median(rel) < 1e-5
        Qf = host(R.apply_operator_block(0.7, V, precision="f32_ir"))
        want_f = op.apply_A_f32(X, 0.7, V.T).T
        bound_f = op.apply_A_f32_bound(X, V.T).T + 1e-12 * np.abs(want_f)
        assert np.all(np.abs(Qf - want_f) <= bound_f), m
    R.close()


def test_dense_autotune(rr, small):
    """The tuned split of the column pass's contraction: one of the
    candidates per operator precision, reused from the cache by a second
    handle of the same shape bucket, and the operator still within the same
    bounds as with the default split."""
    X = small.astype(np.float64)
    R0 = rr.DenseRidge(small)
    assert R0.info["dense_split"] == [1024, 256, 1024]
    R = rr.DenseRidge(small, autotune=True)
    split = R.info["dense_split"]
    assert all(t in (128, 256, 512, 1024, 2048) for t in split), split
    R2 = rr.DenseRidge(small, autotune=True)
    assert R2.info["dense_split_cached"] == 1 and R2.info["dense_split"] == split
    print(f"[dense autotune] split targets {split}", flush=True)
    V = np.random.default_rng(9).standard_normal((37, X.shape[1]))
    Q = host(R.apply_operator_block(0.7, V))
    for c in range(V.shape[0]):
        want = op.apply_A(X, 0.7, V[c])
        bound = 4 * (X.shape[0] + X.shape[1]) * 2.0**-53 * (np.abs(X).T @ (np.abs(X) @ np.abs(V[c])) + 0.7 * np.abs(V[c]))
        assert np.all(np.abs(Q[c] - want) <= bound), c
    Qb = host(R.apply_operator_block(0.7, V, precision="bf16_ir"))
    want_b = op.apply_A_bf16(X, 0.7, V.T).T
    assert np.all(np.abs(Qb - want_b) <= op.apply_A_bf16_bound(X, V.T).T + 1e-12 * np.abs(want_b))
    for h in (R0, R, R2):
        h.close()


def test_operator_lambda_zero_and_zero_block(rr, small):
    R = rr.DenseRidge(small)
    V = np.zeros((3, small.shape[1]))
    assert np.all(host(R.apply_operator_block(0.0, V)) == 0.0)
    V[1, 5] = 1.0
    q = host(R.apply_operator_block(0.0, V))[1]
    X = small.astype(np.float64)
    assert np.allclose(q, X.T @ X[:, 5], rtol=1e-12, atol=1e-9)
    R.close()


@pytest.fixture(scope="module")
def clustered(rr, small):
    lab, fc, _, _ = kmeans.kmeans_features(small.astype(np.float64), 40, 3, binary=False)
    print(f"[dense clustered] F_C={fc}", flush=True)
    R = rr.DenseRidge(small, labels=lab)
    yield small.astype(np.float64), lab, fc, R
    R.close()


def test_coarse_gram_and_weight(rr, clustered):
    X, lab, fc, R = clustered
    assert R.info["n_coarse"] == fc
    assert np.array_equal(host(R.labels()), lab)
    K_or = coarse.coarse_gram(X, lab, fc)
    K = host(R.coarse_gram())
    assert np.abs(K - K_or).max() <= 1e-12 * np.abs(K_or).max()
    for lam in (0.1, 10.0):
        om = R.smoother_weight(lam)
        om_or = op.omega_power(X, lam, seed=0x5eed)
        assert abs(om - om_or) <= 1e-10 * om_or


def oracle_spread(X, b, lam, kind, lab, fc, omega, tol, n=8, seed=0):
    """Iteration counts of the oracle under rounding-level changes: the
    operator through the Gram matrix (another summation order) on odd runs,
    the diagonal (or an identity scaling for CG) perturbed by at most 2 ulp,
    and for the two-level forms also the coarse solve through an explicit
    inverse.  Near a residual plateau the natural stop spans this range."""
    F = X.shape[1]
    rng = np.random.default_rng(seed)
    G = X.T @ X
    its = []
    for t in range(n):
        pert = np.ones(F) if t == 0 else 1.0 + (rng.random(F) - 0.5) * 4 * 2**-53
        A = (lambda v: G @ v + lam * v) if t % 2 else (lambda v: op.apply_A(X, lam, v))
        if kind == "none":
            B = lambda r, pert=pert: r * pert
        elif kind == "jacobi":
            D = op.jacobi_diagonal(X, lam) * pert
            B = lambda r, D=D: r / D
        else:
            tl = precond.TwoLevel(X, lam, lab, fc, omega)
            tl.D = tl.D * pert
            if t == 2:
                Ai = np.linalg.inv(tl.Ac)
                tl.coarse_correction = lambda r, tl=tl, Ai=Ai: tl.P @ (Ai @ (tl.P.T @ r))
            B = tl.vcycle if kind == "vcycle" else tl.additive
        _, inf = krylov.pcg(A, b, B, tol=tol, max_iter=20000)
        its.append(inf.iters)
    return min(its), max(its)


@pytest.mark.parametrize("kind", ["vcycle", "additive", "jacobi", "none"])
def test_block_solve_f64_parity(rr, clustered, kind):
    """(P2) natural stop at relative residual 1e-10: each column's count
    within the oracle's own spread under rounding-level changes, +-1; (P1)
    at the oracle's count for a residual of 1e-12 the block iterate equals
    the oracle's to 1e-10 per column."""
    X, lab, fc, R = clustered
    lam = 0.1
    _, Y = datagen.targets(X, 77, n_rhs=9)
    Y = Y.T.copy()                      # (m, N)
    om = op.omega_power(X, lam, seed=0x5eed)
    tol = 1e-10
    W, infos = R.solve_block(lam, Y, precond=kind, tol=tol, max_iter=20000)
    kfix = 0
    for c in range(Y.shape[0]):
        lo, hi = oracle_spread(X, op.rhs(X, Y[c]), lam, kind, lab, fc, om, tol, seed=c)
        k = infos[c]["iters"]
        print(f"[dense {kind}] col {c}: gpu {k} its, oracle {lo}..{hi}", flush=True)
        assert infos[c]["status"] == 0
        assert lo - 1 <= k <= hi + 1
        assert infos[c]["true_relres"] <= 10 * tol
        _, inf12 = krylov.solve(X, Y[c], lam, kind, lab, fc, omega=om, tol=1e-12, max_iter=20000)
        kfix = max(kfix, inf12.iters)
    W, infos = R.solve_block(lam, Y, precond=kind, fixed_iters=kfix)
    W = host(W)
    for c in range(Y.shape[0]):
        x_or, _ = krylov.solve(X, Y[c], lam, kind, lab, fc, omega=om, fixed_iters=kfix)
        assert infos[c]["iters"] == kfix
        assert np.linalg.norm(W[c] - x_or) <= 1e-10 * np.linalg.norm(x_or), c


def test_block_solve_fixed_iterations(rr, clustered):
    """Three V(1,1) iterations: the GPU iterate is the oracle's up to rounding."""
    X, lab, fc, R = clustered
    lam = 0.1
    _, Y = datagen.targets(X, 78, n_rhs=4)
    Y = Y.T.copy()
    om = op.omega_power(X, lam, seed=0x5eed)
    W, infos = R.solve_block(lam, Y, precond="vcycle", fixed_iters=3)
    W = host(W)
    for c in range(4):
        x_or, inf = krylov.solve(X, Y[c], lam, "vcycle", lab, fc, omega=om, fixed_iters=3)
        assert infos[c]["iters"] == 3
        assert np.linalg.norm(W[c] - x_or) <= 1e-11 * np.linalg.norm(x_or)


def test_block_solve_bf16_refinement(rr, clustered):
    X, lab, fc, R = clustered
    lam = 0.1
    _, Y = datagen.targets(X, 79, n_rhs=6)
    Y = Y.T.copy()
    W, infos = R.solve_block(lam, Y, precond="vcycle", precision="bf16_ir", tol=1e-13)
    W = host(W)
    for c in range(6):
        w_star = krylov.reference_solution(X, Y[c], lam)
        err = np.linalg.norm(W[c] - w_star) / np.linalg.norm(w_star)
        print(f"[dense bf16 IR] col {c}: {infos[c]['ir_steps']} steps, {infos[c]['iters']} its, "
              f"err {err:.2e}", flush=True)
        assert infos[c]["status"] == 0 and infos[c]["ir_steps"] >= 2
        assert err <= 1e-10


def test_block_solve_f32_refinement(rr, clustered):
    X, lab, fc, R = clustered
    lam = 0.1
    _, Y = datagen.targets(X, 81, n_rhs=5)
    Y = Y.T.copy()
    W, infos = R.solve_block(lam, Y, precond="vcycle", precision="f32_ir", tol=1e-13)
    W = host(W)
    for c in range(5):
        w_star = krylov.reference_solution(X, Y[c], lam)
        err = np.linalg.norm(W[c] - w_star) / np.linalg.norm(w_star)
        print(f"[dense f32 IR] col {c}: {infos[c]['ir_steps']} steps, {infos[c]['iters']} its, "
              f"err {err:.2e}", flush=True)
        assert infos[c]["status"] == 0 and infos[c]["ir_steps"] >= 2
        assert err <= 1e-10


def test_block_solve_edges(rr, clustered):
    X, lab, fc, R = clustered
    F = X.shape[1]
    rng = np.random.default_rng(9)
    B = rng.standard_normal((3, F))
    B[1] = 0.0                                   # a zero right-hand side
    W, infos = R.solve_block(1.0, B, rhs_is_b=True, precond="vcycle", tol=1e-13)
    W = host(W)
    assert infos[1]["iters"] == 0 and np.all(W[1] == 0.0)
    A = X.T @ X + np.eye(F)
    for c in (0, 2):
        ref = np.linalg.solve(A, B[c])
        assert np.linalg.norm(W[c] - ref) <= 1e-10 * np.linalg.norm(ref)
    w1, info1 = R.solve(1.0, B[0], rhs_is_b=True, precond="vcycle", tol=1e-13)
    assert np.linalg.norm(host(w1) - W[0]) <= 1e-12 * np.linalg.norm(W[0])


def test_dense_kmeans(rr, small):
    """GPU k-means++ on dense columns against the oracle (FP64 in both, sums
    in different orders): the seeding draws the same centres (a draw would
    differ only if u T fell within rounding of a prefix boundary), the labels
    agree on >= 99 % of the features, and the GPU labels are a Lloyd fixed
    point up to near-ties of the FP64 scores."""
    X = small.astype(np.float64)
    k = 40
    R = rr.DenseRidge(small, n_clusters=k, seed=3)
    assert np.array_equal(host(R.centres()), kmeans.seed_real(X, k, 3))
    lab_or, fc_or, it_or, _ = kmeans.kmeans_features(X, k, 3, binary=False)
    lab = host(R.labels())
    fc = R.info["n_coarse"]
    print(f"[dense kmeans] F_C gpu {fc} oracle {fc_or}, passes gpu {R.info['kmeans_iters']} "
          f"oracle {it_or}, agree {np.mean(lab == lab_or):.4f}", flush=True)
    assert np.mean(lab == lab_or) >= 0.99
    mu = np.stack([X[:, lab == c].mean(axis=1) for c in range(fc)], axis=1)
    score = np.einsum("is,is->s", mu, mu)[None, :] - 2.0 * (X.T @ mu)
    best = np.argmin(score, axis=1)
    rows = np.arange(X.shape[1])
    gap = score[rows, lab] - score[rows, best]
    scale = np.abs(score).max()
    assert np.all(gap <= 1e-9 * scale)
    # the two-level solve on the GPU's own aggregation converges
    _, Y = datagen.targets(X, 80, n_rhs=2)
    W, infos = R.solve_block(0.1, Y.T.copy(), precond="vcycle", tol=1e-10)
    assert all(i["status"] == 0 for i in infos)
    R.close()


def test_dense_errors(rr, small):
    R = rr.DenseRidge(small)
    with pytest.raises(rr.RRError) as e:          # no coarse level
        R.solve_block(1.0, np.ones((1, small.shape[0])), precond="vcycle")
    assert e.value.status == rr.RR_ERR_INVALID_ARG
    with pytest.raises(rr.RRError) as e:          # sparse-only call
        rr.rr_apply_rhs(R.h, torch.zeros(small.shape[0], dtype=torch.float64, device="cuda"),
                        torch.zeros(small.shape[1], dtype=torch.float64, device="cuda"))
    assert e.value.status == rr.RR_ERR_UNSUPPORTED
    bad = small.copy()
    bad[3, 4] = np.nan
    with pytest.raises(rr.RRError) as e:
        rr.DenseRidge(bad)
    assert e.value.status == rr.RR_ERR_INVALID_ARG
    R.close()


@pytest.fixture(scope="module")
def mid(rr):
    """8192 x 2048 (32 groups of 64 columns, correlation 0.9) with 64
    right-hand sides: the column pass's contraction splits into as many
    pieces per output tile as at 50,000 x 4096 (the tiles and the split
    target do not depend on N beyond the piece count), and every GEMM tile
    is full."""
    X = datagen.block_correlated_dense(8192, 32, 64, 0.9, seed=41).astype(np.float32)
    lab = datagen.random_labels(X.shape[1], 64, 5)
    fc = int(lab.max()) + 1
    print(f"[dense mid] X {X.shape}, F_C={fc}", flush=True)
    R = rr.DenseRidge(X, labels=lab)
    yield X.astype(np.float64), lab, fc, R
    R.close()


def test_mid_operator_all_precisions(rr, mid):
    X, lab, fc, R = mid
    V = np.random.default_rng(9).standard_normal((64, X.shape[1]))
    Q = host(R.apply_operator_block(0.1, V))
    want = (X.T @ (X @ V.T)).T + 0.1 * V
    bound = 4 * (X.shape[0] + X.shape[1]) * 2.0**-53 * ((np.abs(X).T @ (np.abs(X) @ np.abs(V.T))).T + 0.1 * np.abs(V))
    assert np.all(np.abs(Q - want) <= bound)
    Qb = host(R.apply_operator_block(0.1, V, precision="bf16_ir"))
    want_b = op.apply_A_bf16(X, 0.1, V.T).T
    assert np.all(np.abs(Qb - want_b) <= op.apply_A_bf16_bound(X, V.T).T + 1e-12 * np.abs(want_b))
    Qf = host(R.apply_operator_block(0.1, V, precision="f32_ir"))
    want_f = op.apply_A_f32(X, 0.1, V.T).T
    assert np.all(np.abs(Qf - want_f) <= op.apply_A_f32_bound(X, V.T).T + 1e-12 * np.abs(want_f))


@pytest.mark.parametrize("precision", ["f64", "bf16_ir", "f32_ir"])
def test_mid_block_solves(rr, mid, precision):
    """64 right-hand sides at lambda = 0.1: FP64 at the oracle's converged
    count (1e-12) equals the oracle's V(1,1) iterate to 1e-10 per column;
    the refinement forms reach the dense Cholesky solution to 1e-10."""
    X, lab, fc, R = mid
    lam = 0.1
    _, Y = datagen.targets(X, 83, n_rhs=64)
    Y = Y.T.copy()
    om = op.omega_power(X, lam, seed=0x5eed)
    cols = (0, 21, 42, 63)
    if precision == "f64":
        ks, refs = [], {}
        for c in cols:
            x_or, inf = krylov.solve(X, Y[c], lam, "vcycle", lab, fc, omega=om, tol=1e-12, max_iter=5000)
            ks.append(inf.iters)
        kfix = max(ks)
        W, infos = R.solve_block(lam, Y, precond="vcycle", fixed_iters=kfix)
        W = host(W)
        for c in cols:
            x_or, _ = krylov.solve(X, Y[c], lam, "vcycle", lab, fc, omega=om, fixed_iters=kfix)
            err = np.linalg.norm(W[c] - x_or) / np.linalg.norm(x_or)
            print(f"[dense mid f64] col {c}: {kfix} its, diff to oracle {err:.1e}", flush=True)
            assert err <= 1e-10
        return
    W, infos = R.solve_block(lam, Y, precond="vcycle", precision=precision, tol=1e-13)
    W = host(W)
    for c in cols:
        w_star = krylov.reference_solution(X, Y[c], lam)
        err = np.linalg.norm(W[c] - w_star) / np.linalg.norm(w_star)
        print(f"[dense mid {precision}] col {c}: {infos[c]['ir_steps']} steps, {infos[c]['iters']} its, "
              f"err {err:.2e}", flush=True)
        assert infos[c]["status"] == 0 and err <= 1e-10
