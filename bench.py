"""Benchmark: time to 1e-10 relative error of the two-level PCG solve on the
binary fingerprint workload (200,000 x 100,000, 60 nonzeros per row, Zipf(1.1)
column popularity, 12.0 M nonzeros), lambda in {1e-2, 1, 100}, k-means
aggregation with k = 1000, FP64 throughout.

One step = the three solves, each run for the number of iterations at which
its iterate first reaches relative error <= 1e-10 against the CPU oracle's
solution on the same aggregation (the oracle's FP64 V(1,1) PCG with the
GPU's k-means labels, converged to relative residual 1e-13; calibrated before
the timed region).  Setup (transpose, k-means, coarse Gram) and the
per-lambda coarse factorizations are timed separately and reported beside the
step.  The oracle's reference solves are timed on one host thread and give
the CPU baseline.

Prints ONE JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-1e-10 rel. error (s) + SpMV HBM GB/s; batched/BF16/learned vs plain"
HBM_PEAK_GBS = 8000.0


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "operator_binary_200kx100k_traffic.md")
CSRC = os.path.join(ROOT, "paper_1806_05826_amd", "csrc")
# the kernels of one operator application (0/1 X) and their sources
APPLY_KERNELS = ("k_rows", "k_sell<1>", "k_sell_reduce<2>")
APPLY_SOURCES = ("rows.hip", "sell.hip", "rr_device.h")


def column_gather_bytes(N, F, nnz):
    """Algorithmic bytes of the column-pass gather t = X^T u (0/1 X): the CSC
    pattern (4-byte row indexes, column pointers), u read once, t written."""
    return 4 * nnz + 4 * (F + 1) + 8 * N + 8 * F


def apply_bytes(N, F, nnz):
    """One operator application q = X^T (X p) + lambda p with the pattern
    stored both ways: both index arrays and pointer arrays, p read twice, u
    written and read, q written."""
    return 8 * nnz + 4 * (N + 1) + 4 * (F + 1) + 8 * F * 2 + 16 * N + 8 * F


def apply_bytes_valued(N, F, nnz):
    """One application with FP64 values stored both ways: 12 bytes per entry
    per pass (4-byte index, 8-byte value) on top of the pattern's vectors."""
    return apply_bytes(N, F, nnz) + 16 * nnz


def sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in APPLY_SOURCES:
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes of one operator application (row pass, column gather,
    column reduction) from the committed counter summary, or None when it is
    missing or was taken on a different version of the kernels' sources."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            fields[k.strip()] = v.strip().strip("`")
    try:
        if fields.get("sources sha256") != sources_hash():
            return None
        return float(fields["apply HBM bytes"])
    except (KeyError, ValueError, OSError):
        return None


def oracle_reference(X, y, lams, labels, fc, log):
    """The oracle's V(1,1) two-level PCG (FP64 SciPy/NumPy, BLAS held to one
    thread) on the GPU's aggregation, run to relative residual 1e-13 per
    lambda: its solution is the reference w*, and its time per iteration
    gives the CPU baseline."""
    from threadpoolctl import threadpool_limits
    from oracle import krylov, operator as op, precond
    out = {}
    with threadpool_limits(limits=1):
        b = op.rhs(X, y)
        for lam in lams:
            omega = op.omega_gershgorin(X, lam)
            B, _ = precond.make("vcycle", X, lam, labels, fc, omega)
            A = lambda v, lam=lam: op.apply_A(X, lam, v)
            t0 = time.perf_counter()
            x, inf = krylov.pcg(A, b, B, tol=1e-13, max_iter=400)
            dt = time.perf_counter() - t0
            k10 = next((k for k, h in enumerate(inf.history) if h <= 1e-10), None)
            out[lam] = {"w": x, "iters": inf.iters, "iters_relres_1e-10": k10, "s": dt,
                        "s_per_iter": dt / max(1, inf.iters), "true_relres": inf.true_relres}
            log(f"[bench oracle] lambda={lam}: {inf.iters} iterations to relres 1e-13 in {dt:.1f} s "
                f"(relres 1e-10 at iteration {k10}), true relres {inf.true_relres:.1e}")
    return out


def valued_operator_section(rr, torch, dev, log, P):
    """The operator of the same 0/1 matrix stored with FP64 values (CSR and
    CSC with 8-byte values: 294.8 MB per application, larger than the 256 MB
    Infinity Cache): 50 back-to-back applications timed with HIP events on
    the current stream."""
    N, F = P.X.shape
    nnz = P.X.nnz
    R = rr.Ridge(P.X, n_clusters=0, binary=False)
    v = torch.randn(F, dtype=torch.float64, device=dev, generator=torch.Generator(device=dev).manual_seed(3))
    out = torch.empty_like(v)
    for _ in range(5):
        rr.rr_apply_operator(R.h, 1.0, v, out)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = 50
    e0.record()
    for _ in range(reps):
        rr.rr_apply_operator(R.h, 1.0, v, out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    R.close()
    b = apply_bytes_valued(N, F, nnz)
    gbs = b / (ms * 1e-3) / 1e9
    log(f"[bench valued] FP64-valued operator: {ms * 1e3:.1f} us per application, {gbs:.0f} GB/s "
        f"({gbs / HBM_PEAK_GBS:.3f} of HBM peak)")
    return {"apply_bytes": b, "apply_ms": ms, "apply_gbs": gbs, "frac": gbs / HBM_PEAK_GBS,
            "kernels": "rr::k_rows_val (row pass: hot values against the LDS slice of v, cold "
                       "ones gathered), rr::k_sell_val<1> (sliced column gather with the values "
                       "streamed beside the 16-bit indexes), rr::k_sell_reduce (column sums and "
                       "epilogue), and the gathers between the caller's and the internal feature "
                       "order"}


def dense_section(rr, torch, dev, log):
    """Dense correlated features with many right-hand sides: X 50,000 x 4096
    FP32, 64 groups of 64 columns with correlation 0.9, 256 targets,
    lambda = 0.1, k-means k = 128.  Times the block V(1,1) solve to relative
    error <= 1e-10 per column against a reference converged to 1e-13, in
    FP64 and as BF16-operand refinement, and the operator's matrix-core
    GEMMs (4 N F m flops per block application) in BF16, FP32 and FP64."""
    import numpy as np
    import datagen
    N, F, m, lam, k = 50_000, 4096, 256, 0.1, 128
    t0 = time.perf_counter()
    X = datagen.block_correlated_dense(N, 64, 64, 0.9, seed=5826 + 3000)
    _, Y = datagen.targets(X, 5826 + 3000, n_rhs=m)
    gen_s = time.perf_counter() - t0
    R = rr.DenseRidge(X, n_clusters=k, seed=5826, autotune=True)
    del X
    sinfo = R.info
    log(f"[bench dense] data {N}x{F}, {m} rhs (generated in {gen_s:.1f} s); setup "
        f"{sinfo['setup_ms']:.0f} ms (k-means {sinfo['kmeans_ms']:.0f} ms, "
        f"{sinfo['kmeans_iters']} passes), F_C={sinfo['n_coarse']}, tuned split targets "
        f"(f64, bf16, f32) {sinfo['dense_split']}")
    Yd = torch.as_tensor(np.ascontiguousarray(Y.T), dtype=torch.float64, device=dev)
    del Y
    Wref, inf_ref = R.solve_block(lam, Yd, precond="vcycle", tol=1e-13, max_iter=3000)
    ref_n = torch.linalg.norm(Wref, dim=1)

    def run(**kw):
        torch.cuda.synchronize()
        ta = time.perf_counter()
        W, infos = R.solve_block(lam, Yd, **kw)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - ta) * 1e3
        err = float((torch.linalg.norm(W - Wref, dim=1) / ref_n).max())
        its = [i["iters"] for i in infos]
        return {"ms": ms, "max_err": err, "max_iters": max(its), "mean_iters": sum(its) / len(its),
                "ir_steps": max(i["ir_steps"] for i in infos),
                "status_ok": all(i["status"] == 0 for i in infos)}

    forms = {}
    # relative residual 1e-12 leaves relative errors below 1e-10 on this matrix
    forms["vcycle_f64"] = run(precond="vcycle", tol=1e-12, max_iter=3000)
    forms["vcycle_bf16_ir"] = run(precond="vcycle", precision="bf16_ir", tol=1e-12, max_iter=3000)
    forms["vcycle_f32_ir"] = run(precond="vcycle", precision="f32_ir", tol=1e-12, max_iter=3000)
    forms["jacobi_f64"] = run(precond="jacobi", tol=1e-12, max_iter=3000)
    forms["jacobi_bf16_ir"] = run(precond="jacobi", precision="bf16_ir", tol=1e-12, max_iter=3000)
    for name, f in forms.items():
        log(f"[bench dense] {name}: {f['ms']:.1f} ms, {f['max_iters']} its (max), "
            f"{f['ir_steps']} IR steps, max rel. error {f['max_err']:.2e}")
    # operator timing: one block application (both GEMMs and the sum)
    V = torch.randn(m, F, dtype=torch.float64, device=dev)
    Q = torch.empty_like(V)
    gemm = {}
    for prec, peak in (("bf16_ir", 2500.0), ("f32_ir", 157.3), ("f64", 78.6)):
        for _ in range(2):
            rr.rr_apply_operator_block(R.h, lam, V, Q, prec)
        reps = {"bf16_ir": 20, "f32_ir": 10}.get(prec, 5)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            rr.rr_apply_operator_block(R.h, lam, V, Q, prec)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        tf = 4.0 * N * F * m / (ms * 1e-3) / 1e12
        gemm[prec] = {"ms_per_apply": ms, "tflops": tf, "peak_tflops": peak, "frac": tf / peak}
        log(f"[bench dense] operator {prec}: {ms:.3f} ms per block apply, {tf:.1f} TFLOP/s "
            f"({100 * tf / peak:.1f} % of {peak} TFLOP/s)")
    R.close()
    return {"workload": f"dense {N}x{F} FP32, 64 groups x 64 columns (correlation 0.9), {m} rhs, "
                        f"lambda={lam}, k-means k={k}",
            "setup_ms": sinfo["setup_ms"], "kmeans_ms": sinfo["kmeans_ms"],
            "n_coarse": sinfo["n_coarse"], "ref_iters": max(i["iters"] for i in inf_ref),
            "split_targets_f64_bf16_f32": sinfo["dense_split"],
            "forms": forms, "operator": gemm}


def bayes_section(rr, torch, dev, log, P, R, k, n_samples=100):
    """Noise-injection samples of Bayesian regression (eq. ni_xtx) on the
    200,000 x 100,000 workload: every sample draws standard normals xi1 (N),
    xi2 (F) and a precision ratio beta = lambda / tau (log-uniform in [0.5, 2],
    a new value each sample as in a Gibbs sweep), forms b = X^T (y + e1) +
    e2 / tau on the GPU and solves (X^T X + beta I) w = b by V(1,1) PCG to
    relative residual 1e-8.  The handle with the eigen coarse solver (K =
    Q diag(ev) Q^T once, one GEMM per beta) against the bench's Cholesky
    handle (a factorization per beta)."""
    import numpy as np
    t0 = time.perf_counter()
    RE = rr.Ridge(P.X, n_clusters=k, seed=5826, lambda_slots=4, coarse_eigen=True)
    torch.cuda.synchronize()
    eig_setup_ms = (time.perf_counter() - t0) * 1e3
    N, F = P.X.shape
    rng = np.random.default_rng(5826 + 5000)
    betas = np.exp(rng.uniform(np.log(0.5), np.log(2.0), n_samples))
    taus = np.exp(rng.uniform(np.log(0.5), np.log(2.0), n_samples))
    g = torch.Generator(device=dev).manual_seed(5826 + 5001)
    y = torch.as_tensor(P.y, dtype=torch.float64, device=dev)
    xi1 = torch.randn((n_samples, N), dtype=torch.float64, device=dev, generator=g)
    xi2 = torch.randn((n_samples, F), dtype=torch.float64, device=dev, generator=g)
    b = torch.empty(F, dtype=torch.float64, device=dev)
    w = torch.empty(F, dtype=torch.float64, device=dev)
    out = {"samples": n_samples, "tol": 1e-8, "eigen_setup_ms": eig_setup_ms,
           "eigen_sweeps": RE.info["eigen_sweeps"]}
    for name, H in (("eigen", RE), ("cholesky", R)):
        iters = []
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for i in range(n_samples):
            tau = float(taus[i])
            lam = float(betas[i]) * tau
            rr.rr_noise_rhs(H.h, tau, lam, y, xi1[i], xi2[i], b)
            st, inf = rr.rr_solve(H.h, lam / tau, b, w, rhs_is_b=True, tol=1e-8, precond="vcycle",
                                  max_iter=5000, raise_on=(1, 2, 6))
            iters.append(inf["iters"])
        torch.cuda.synchronize()
        ms = (time.perf_counter() - ta) * 1e3
        out[name] = {"ms_per_sample": ms / n_samples, "mean_iters": float(np.mean(iters))}
    RE.close()
    log(f"[bench bayes] {n_samples} noise-injection samples, beta in [0.5, 2]: eigen coarse "
        f"{out['eigen']['ms_per_sample']:.2f} ms/sample ({out['eigen']['mean_iters']:.1f} its; "
        f"decomposition in setup {eig_setup_ms:.0f} ms, {out['eigen_sweeps']} Jacobi sweeps), "
        f"Cholesky per beta {out['cholesky']['ms_per_sample']:.2f} ms/sample "
        f"({out['cholesky']['mean_iters']:.1f} its)")
    return out


def newton_section(rr, torch, dev, log, P, k, steps=5, beta=1.0):
    """L2-regularized logistic regression on the 200,000 x 100,000 matrix
    (targets t = 1[y > median y]) by Newton steps: each step forms z = X w,
    p = sigma(z), the gradient g = X^T (p - t) + beta w, sets the row weights
    d = p (1 - p) (which rebuilds the Jacobi diagonal, the Gershgorin sums
    and the coarse matrix P^T X^T D X P) and solves (X^T D X + beta I) s = -g
    by V(1,1) PCG to relative residual 1e-8 (the Hessian form of the
    subsection on optimization by the Newton method)."""
    import numpy as np
    R = rr.Ridge(P.X, n_clusters=k, seed=5826, lambda_slots=4)   # no block-smoother blocks
    N, F = P.X.shape
    y = np.asarray(P.y)
    t = torch.as_tensor((y > np.median(y)).astype(np.float64), device=dev)
    w = torch.zeros(F, dtype=torch.float64, device=dev)
    s = torch.empty(F, dtype=torch.float64, device=dev)
    rows = []
    for k in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        z = R.apply_rows(w)
        p = torch.sigmoid(z)
        g = R.apply_rhs(p - t) + beta * w
        loss = float((torch.nn.functional.softplus(z) - t * z).sum() + 0.5 * beta * (w * w).sum())
        gnorm = float(g.norm())
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        R.set_row_weights(p * (1.0 - p))
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        st, inf = rr.rr_solve(R.h, beta, -g, s, rhs_is_b=True, tol=1e-8, precond="vcycle",
                              max_iter=5000, raise_on=(1, 2, 6))
        w += s
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        rows.append({"loss": loss, "grad_norm": gnorm, "iters": inf["iters"],
                     "gradient_ms": (t1 - t0) * 1e3, "weights_ms": (t2 - t1) * 1e3,
                     "solve_ms": (t3 - t2) * 1e3})
    R.close()
    log("[bench newton] " + "; ".join(
        f"step {i}: loss {r['loss']:.6e}, |g| {r['grad_norm']:.2e}, {r['iters']} its, weights "
        f"{r['weights_ms']:.1f} ms, solve {r['solve_ms']:.1f} ms" for i, r in enumerate(rows)))
    return {"steps": rows, "beta": beta, "tol": 1e-8}


def tiny_section(rr, torch, dev, log, reps=20):
    """The tiny plain-method workload (2000 x 500 binary, 2 % density,
    Zipf(1.1) columns, lambda = 1, k-means k = 50): unpreconditioned CG
    against Jacobi PCG and the two-level forms, each to relative residual
    1e-10; iterations, time per solve (mean of `reps`, after one warm-up)
    and the relative error against a dense Cholesky solve of the normal
    equations (NumPy, FP64)."""
    import numpy as np
    import datagen
    P = datagen.tiny_sparse()
    lam = 1.0
    Xd = P.X.toarray()
    A = Xd.T @ Xd + lam * np.eye(Xd.shape[1])
    L = np.linalg.cholesky(A)
    wx = np.linalg.solve(L.T, np.linalg.solve(L, Xd.T @ P.y))
    R = rr.Ridge(P.X, n_clusters=50, seed=5826)
    y = torch.as_tensor(P.y, dtype=torch.float64, device=dev)
    w = torch.empty(P.X.shape[1], dtype=torch.float64, device=dev)
    out = {"workload": "binary 2000x500, 10 nnz/row, Zipf(1.1) columns, lambda=1, k-means k=50, "
                       "stop at relative residual 1e-10",
           "n_coarse": R.info["n_coarse"], "forms": {}}
    for kind in ("none", "jacobi", "vcycle", "additive"):
        rr.rr_solve(R.h, lam, y, w, tol=1e-10, max_iter=5000, precond=kind, raise_on=(1, 2, 6))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            st, inf = rr.rr_solve(R.h, lam, y, w, tol=1e-10, max_iter=5000, precond=kind,
                                  raise_on=(1, 2, 6))
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        err = float(np.linalg.norm(w.cpu().numpy() - wx) / np.linalg.norm(wx))
        out["forms"][kind] = {"iters": inf["iters"], "ms": ms, "err": err,
                              "true_relres": inf["true_relres"]}
        log(f"[bench tiny] {kind}: {inf['iters']} iterations, {ms:.3f} ms, rel. error {err:.2e}")
    R.close()
    return out


def leader_section(rr, torch, dev, log, P, R, tol=24.0):
    """Leader-follower aggregation (the paper's experiments' clustering) on
    the 200,000 x 100,000 workload at distance tolerance `tol`, against the
    bench's k-means (k = 1000) handle: V(1,1) PCG to relative residual 1e-10
    at each lambda, iterations and time per solve."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    RL = rr.Ridge(P.X, lf_tolerance=tol, lambda_slots=4)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    y = torch.as_tensor(P.y, dtype=torch.float64, device=dev)
    w = torch.empty(P.X.shape[1], dtype=torch.float64, device=dev)
    out = {"tolerance": tol, "n_coarse": RL.info["n_coarse"], "setup_ms": setup_ms,
           "clustering_ms": RL.info["kmeans_ms"], "per_lambda": {}}
    for lam in (1e-2, 1.0, 100.0):
        row = {}
        for name, H in (("leader_follower", RL), ("kmeans", R)):
            rr.rr_solve(H.h, lam, y, w, tol=1e-10, precond="vcycle", max_iter=5000, raise_on=(1, 2, 6))
            torch.cuda.synchronize()
            ta = time.perf_counter()
            st, inf = rr.rr_solve(H.h, lam, y, w, tol=1e-10, precond="vcycle", max_iter=5000, raise_on=(1, 2, 6))
            torch.cuda.synchronize()
            row[name] = {"iters": inf["iters"], "ms": (time.perf_counter() - ta) * 1e3}
        out["per_lambda"][str(lam)] = row
    out["least_squares"] = ls_interp_part(rr, torch, dev, RL, y, w)
    RL.close()
    log(f"[bench leader] tolerance {tol}: F_C={out['n_coarse']}, clustering {out['clustering_ms']:.0f} ms; " +
        "; ".join(f"lambda={l}: LF {r['leader_follower']['iters']} its {r['leader_follower']['ms']:.1f} ms, "
                  f"k-means {r['kmeans']['iters']} its {r['kmeans']['ms']:.1f} ms"
                  for l, r in out["per_lambda"].items()))
    ls = out["least_squares"]
    log(f"[bench leader] least-squares interpolation ({ls['prototypes']} principal components): " +
        "; ".join(f"lambda={l}: {r['iters']} its {r['ms']:.1f} ms (weights + coarse Gram {r['set_ms']:.0f} ms)"
                  for l, r in ls["per_lambda"].items()))
    return out


def ls_interp_part(rr, torch, dev, RL, y, w, n_proto=8, steps=40):
    """Least-squares interpolation on the leader-follower aggregation of
    RL.  The prototypes are the n_proto leading principal components of
    X^T X from rr_prototypes (`steps` Lanczos steps with full
    reorthogonalisation on the GPU), before any timing; rr_set_interpolation
    then runs at beta = lambda for every lambda, and a V(1,1) PCG solve to
    relative residual 1e-10 follows."""
    import numpy as np
    F = RL.F
    V = torch.empty((n_proto, F), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev = rr.rr_prototypes(RL.h, n_proto, V, steps=steps)
    torch.cuda.synchronize()
    proto_ms = (time.perf_counter() - t0) * 1e3
    Q = V.t().contiguous().cpu().numpy()
    out = {"prototypes": n_proto, "lanczos_steps": steps, "prototype_ms": proto_ms,
           "ritz_values": [float(x) for x in ev], "per_lambda": {}}
    for lam in (1e-2, 1.0, 100.0):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        RL.set_interpolation(Q, lam)
        torch.cuda.synchronize()
        set_ms = (time.perf_counter() - t0) * 1e3
        rr.rr_solve(RL.h, lam, y, w, tol=1e-10, precond="vcycle", max_iter=5000, raise_on=(1, 2, 6))
        torch.cuda.synchronize()
        ta = time.perf_counter()
        st, inf = rr.rr_solve(RL.h, lam, y, w, tol=1e-10, precond="vcycle", max_iter=5000, raise_on=(1, 2, 6))
        torch.cuda.synchronize()
        out["per_lambda"][str(lam)] = {"iters": inf["iters"], "ms": (time.perf_counter() - ta) * 1e3,
                                       "set_ms": set_ms, "converged": bool(inf["status"] == 0)}
    RL.set_interpolation(None)
    return out


def batched_uneven_section(rr, torch, dev, log, full=True):
    """Independent uneven problems: the batched-uneven workload's generator
    (binary entries, density 1-5 %, Zipf columns, lambda log-uniform in
    [1e-3, 10], k = ceil(d / 10) clamped to [8, 800], relative residual 1e-8),
    by default the whole workload: 500 problems, n in [500, 20000], d in
    [200, 8000]; with ``full`` False 100 problems at n in [500, 5000] and d
    in [200, 2000].  Times every problem in one persistent kernel launch
    (replayed from a HIP graph) against the stream form of rr_solve_batched
    (a work set and a stream per problem, iteration chunks replayed from HIP
    graphs) and, for the small batch, one rr_solve after another."""
    import numpy as np
    import datagen
    n_problems, n_range, d_range = (500, (500, 20_000), (200, 8_000)) if full else \
        (100, (500, 5000), (200, 2000))
    t0 = time.perf_counter()
    batch = datagen.batched_problems(n_problems, seed=5826 + 4000, n_range=n_range, d_range=d_range,
                                     workers=min(16, os.cpu_count() or 1) if full else 1)
    gen_s = time.perf_counter() - t0
    nnz = int(sum(P.X.nnz for P, _ in batch))
    log(f"[bench batched] generated {n_problems} problems, {nnz / 1e6:.1f} M nnz in {gen_s:.1f} s")
    t0 = time.perf_counter()
    Rs, rhs, ws, lams = [], [], [], []
    for i, (P, lam) in enumerate(batch):
        k = int(min(800, max(8, -(-P.X.shape[1] // 10))))
        Rs.append(rr.Ridge(P.X, n_clusters=k, seed=9, autotune=True))
        rhs.append(torch.as_tensor(P.y, dtype=torch.float64, device=dev))
        ws.append(torch.empty(P.X.shape[1], dtype=torch.float64, device=dev))
        lams.append(lam)
        if (i + 1) % 100 == 0:
            log(f"[bench batched] set up {i + 1} problems ({time.perf_counter() - t0:.1f} s)")
    shapes = [(P.X.shape[0], P.X.shape[1], P.X.nnz) for P, _ in batch]
    del batch
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    hs = [R.h for R in Rs]
    kw = dict(tol=1e-8, precond="vcycle", max_iter=5000)

    def timed(f):
        torch.cuda.synchronize()
        ta = time.perf_counter()
        r = f()
        torch.cuda.synchronize()
        return r, (time.perf_counter() - ta) * 1e3

    # warm-up (per-lambda coarse factors are then cached, the launch graph captured)
    rr.rr_solve_batched(hs, lams, rhs, ws, persistent=True, graph=True, **kw)
    (st_p, inf_p), pers_ms = timed(lambda: rr.rr_solve_batched(hs, lams, rhs, ws, persistent=True,
                                                               graph=True, **kw))
    log(f"[bench batched] persistent launch: {pers_ms:.1f} ms")
    hkw = dict(persistent="hybrid", graph=True, chunk=16, **kw)
    rr.rr_solve_batched(hs, lams, rhs, ws, **hkw)
    (st_h, inf_h), hyb_ms = timed(lambda: rr.rr_solve_batched(hs, lams, rhs, ws, **hkw))
    # the caps of the hybrid form (as the library computes them): problems
    # whose count passed their cap continued on the streams
    cost = [n + d + z for n, d, z in shapes]
    grid0 = min(n_problems, torch.cuda.get_device_properties(0).multi_processor_count)
    bud = 512.0 * sum(cost) / grid0
    caps = [max(16, int(np.ceil(bud / c))) for c in cost]
    handed = sum(1 for i, inf in enumerate(inf_h) if inf["iters"] > caps[i])
    log(f"[bench batched] hybrid launch + stream continuation: {hyb_ms:.1f} ms "
        f"({handed} problems continued on the streams)")
    rr.rr_solve_batched(hs, lams, rhs, ws, chunk=16, graph=True, **kw)
    (st_g, inf_g), graph_ms = timed(lambda: rr.rr_solve_batched(hs, lams, rhs, ws, chunk=16, graph=True,
                                                                **kw))
    log(f"[bench batched] stream work sets with graph replay: {graph_ms:.1f} ms")
    seq_ms = None
    if not full:
        def seq():
            return [rr.rr_solve(h, lam, b, w, raise_on=(1, 2, 6), **kw)[1]["iters"]
                    for h, lam, b, w in zip(hs, lams, rhs, ws)]
        seq()
        _, seq_ms = timed(seq)
    ok = st_p == 0 and st_g == 0 and st_h == 0 and all(i["status"] == 0 for i in inf_p + inf_g + inf_h)
    it_h = [i["iters"] for i in inf_h]
    it_p = [i["iters"] for i in inf_p]
    it_g = [i["iters"] for i in inf_g]
    # the two paths add in different orders: iteration counts at the natural
    # stop agree within 1 + 2 %
    outside = sum(1 for a, b in zip(it_p, it_g) if abs(a - b) > 1 + 0.02 * b)
    outside_h = sum(1 for a, b in zip(it_h, it_g) if abs(a - b) > 1 + 0.02 * b)
    worst = max(range(n_problems), key=lambda i: abs(it_h[i] - it_g[i]))
    for R in Rs:
        R.close()
    # the persistent launch's schedule: each problem's time on its workgroup
    # (rr_solve_info.ms), the busy fraction of the workgroups over the launch
    # and the longest problems
    busy = [i["ms"] for i in inf_p]
    grid = min(n_problems, torch.cuda.get_device_properties(0).multi_processor_count)
    util = sum(busy) / (grid * pers_ms)
    top = sorted(range(n_problems), key=lambda i: -busy[i])[:5]
    log(f"[bench batched] persistent: workgroups busy {100 * util:.0f} % of the launch; longest problems "
        + ", ".join(f"{busy[i]:.0f} ms ({it_p[i]} it, {shapes[i][0]}x{shapes[i][1]}, "
                    f"{shapes[i][2] / 1e6:.2f} M nnz)" for i in top))
    log(f"[bench batched] {n_problems} problems, {nnz / 1e6:.1f} M nnz (generated {gen_s:.1f} s, "
        f"setup {setup_s:.1f} s): persistent {pers_ms:.1f} ms, hybrid {hyb_ms:.1f} ms, stream+graphs "
        f"{graph_ms:.1f} ms (hybrid {graph_ms / hyb_ms:.2f}x of stream+graphs), all converged {ok}; "
        f"iteration counts outside 1 + 2 % of the stream form's: persistent {outside}, hybrid "
        f"{outside_h} (largest: {it_g[worst]} -> {it_h[worst]} at {shapes[worst][0]}x{shapes[worst][1]}, "
        f"lambda {lams[worst]:.2e})")
    out = {"problems": n_problems, "nnz": nnz, "n_range": list(n_range), "d_range": list(d_range),
           "tol": 1e-8, "setup_s": setup_s, "persistent_ms": pers_ms, "batched_graph_ms": graph_ms,
           "persistent_vs_graph": graph_ms / pers_ms, "hybrid_ms": hyb_ms,
           "hybrid_vs_graph": graph_ms / hyb_ms, "hybrid_continued": handed, "all_converged": ok,
           "iterations_outside_band": {"persistent": outside, "hybrid": outside_h},
           "largest_iteration_difference": [it_g[worst], it_h[worst]], "total_iters": int(sum(it_p)),
           "max_iters": int(max(it_p)), "persistent_busy_fraction": util,
           "persistent_longest_ms": [busy[i] for i in top]}
    if seq_ms is not None:
        out["sequential_ms"] = seq_ms
        out["persistent_vs_sequential"] = seq_ms / pers_ms
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--k", type=int, default=1000)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="end with a plain 256 MiB device copy (scale for memory counters)")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched uneven-problem section (500 problems up to "
                         "20000 x 8000)")
    ap.add_argument("--batched-small", action="store_true",
                    help="run the batched uneven-problem section on 100 problems up to 5000 x 2000")
    ap.add_argument("--no-dense", action="store_true",
                    help="skip the dense many-rhs and batched uneven-problem sections")
    ap.add_argument("--dense-only", action="store_true",
                    help="run only the dense many-rhs section and print its JSON")
    ap.add_argument("--tiny-only", action="store_true",
                    help="run only the tiny plain-method section (CG against the two-level forms)")
    ap.add_argument("--operator-only", action="store_true",
                    help="run only the timed step at C2, the operator's timing and the FP64-valued "
                         "operator, and print their JSON (for profiler and counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU row-sharded design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import datagen
    import paper_1806_05826_amd as rr

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    if args.dense_only:
        print(json.dumps({"dense_many_rhs": dense_section(rr, torch, dev, log)}), flush=True)
        return
    if args.tiny_only:
        print(json.dumps({"tiny_plain": tiny_section(rr, torch, dev, log)}), flush=True)
        return
    if args.batched_only:
        print(json.dumps({"batched_uneven": batched_uneven_section(rr, torch, dev, log,
                                                                   full=not args.batched_small)}),
              flush=True)
        return
    P = datagen.chembl_like()
    N, F = P.X.shape
    nnz = P.X.nnz
    lams = [1e-2, 1.0, 100.0]
    print(f"[bench] data {N}x{F} nnz={nnz}", file=sys.stderr, flush=True)

    R = rr.Ridge(P.X, n_clusters=args.k, seed=5826, lambda_slots=4, autotune=True, block_smoother=True)
    sinfo = R.info
    print(f"[bench] setup {sinfo['setup_ms']:.0f} ms (k-means {sinfo['kmeans_ms']:.0f} ms, "
          f"{sinfo['kmeans_iters']} Lloyd passes), F_C={sinfo['n_coarse']}", file=sys.stderr, flush=True)
    y = torch.as_tensor(P.y, dtype=torch.float64, device=dev)
    w = torch.empty(F, dtype=torch.float64, device=dev)

    # calibration: the oracle's solution on the GPU's aggregation is the
    # reference; each lambda's fixed count is the GPU's first iteration within
    # 1e-10 relative error of it (with --no-cpu the GPU's own solve to 1e-14
    # serves as the reference instead)
    calib = {}
    wrefs = {}
    orc = None
    if not args.no_cpu:
        labels = R.labels().cpu().numpy()
        orc = oracle_reference(P.X, P.y, lams, labels, sinfo["n_coarse"], log)
    for lam in lams:
        if orc is not None:
            wref = torch.as_tensor(orc[lam]["w"], dtype=torch.float64, device=dev)
            st, inf_ref = rr.rr_solve(R.h, lam, y, w, tol=1e-13, max_iter=3000, precond="vcycle",
                                      raise_on=(1, 2, 6))
        else:
            st, inf_ref = rr.rr_solve(R.h, lam, y, w, tol=1e-14, max_iter=3000, precond="vcycle",
                                      raise_on=(1, 2, 6))
            wref = w.clone()
        wrefs[lam] = wref
        st, inf = rr.rr_solve(R.h, lam, y, w, tol=1e-300, x_ref=wref, err_tol=1e-10,
                              max_iter=3000, precond="vcycle", raise_on=(1, 2, 6))
        calib[lam] = {"iters": inf["iters"], "err": inf["err"], "ref_iters": inf_ref["iters"],
                      "ref_true_relres": inf_ref["true_relres"], "coarse_ms": inf_ref["coarse_ms"]}
        if orc is not None:
            calib[lam]["oracle_iters_to_relres_1e-10"] = orc[lam]["iters_relres_1e-10"]
            calib[lam]["gpu_iters_to_relres_1e-10"] = rr.rr_solve(
                R.h, lam, y, w, tol=1e-10, max_iter=3000, precond="vcycle", raise_on=(1, 2, 6))[1]["iters"]
        print(f"[bench] lambda={lam}: {inf['iters']} iterations to rel. error {inf['err']:.2e} "
              f"against the {'oracle' if orc is not None else 'GPU'} reference",
              file=sys.stderr, flush=True)

    def step(profile=0):
        out = {}
        for lam in lams:
            st, inf = rr.rr_solve(R.h, lam, y, w, fixed_iters=calib[lam]["iters"],
                                  precond="vcycle", profile=profile, chunk=16,
                                  raise_on=(1, 2, 6))
            out[lam] = inf
        return out

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        last = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    # the timed solves' iterates against the reference
    err_final = {}
    for lam in lams:
        rr.rr_solve(R.h, lam, y, w, fixed_iters=calib[lam]["iters"], precond="vcycle", chunk=16,
                    raise_on=(1, 2, 6))
        err_final[lam] = float(torch.linalg.norm(w - wrefs[lam]) / torch.linalg.norm(wrefs[lam]))
    # kernel timing with HIP events recorded by the library on its stream
    prof = step(profile=2)
    prof3 = step(profile=3)
    torch.cuda.synchronize()
    # inside the timed solves: events around each pass (the gaps between
    # kernels that the events force included)
    csc_ms = np.mean([prof[l]["csc_avg_ms"] for l in lams])
    csr_ms = np.mean([prof[l]["csr_avg_ms"] for l in lams])
    # back-to-back launches on the solve's stream (20 each, HIP events around
    # the batch): the row pass, the column gather, and the column gather with
    # its reduction; the last two make one application, the kernels'
    # durations the kernel trace reports
    gcsc_ms = np.mean([prof[l]["csc_gather_avg_ms"] for l in lams])
    gcsr_ms = np.mean([prof3[l]["csr_gather_avg_ms"] for l in lams])
    col_ms = np.mean([prof3[l]["csc_gather_avg_ms"] for l in lams])
    apply_ms = gcsr_ms + col_ms
    b_gather = column_gather_bytes(N, F, nnz)
    gbs_gather = b_gather / (gcsc_ms * 1e-3) / 1e9
    b_apply = apply_bytes(N, F, nnz)
    gbs_op = b_apply / (apply_ms * 1e-3) / 1e9
    # the HBM-resident case: the same matrix with FP64 values stored both ways
    # (295 MB per application, more than the 256 MB Infinity Cache)
    valued = valued_operator_section(rr, torch, dev, log, P)
    if args.operator_only:
        print(json.dumps({"ms_per_step": ms_per_step, "per_lambda_iters": {str(l): calib[l]["iters"] for l in lams},
                          "operator": {"apply_bytes": b_apply, "apply_ms": apply_ms,
                                       "apply_gbs": gbs_op, "row_pass_ms": gcsr_ms,
                                       "column_pass_ms": col_ms, "column_gather_ms": gcsc_ms,
                                       "in_solve_row_pass_ms": csr_ms,
                                       "in_solve_column_pass_ms": csc_ms},
                          "operator_valued_f64": valued}), flush=True)
        if args.calibrate_copy:
            calibration_copy(torch, dev)
        return

    # other forms for comparison (untimed calibration, one timed solve each)
    compare = {}
    for name, kind, sm in (("jacobi", "jacobi", "point"), ("additive", "additive", "point"),
                           ("vcycle_block", "vcycle", "block"), ("additive_block", "additive", "block")):
        lam = 1.0
        st, inf = rr.rr_solve(R.h, lam, y, w, tol=1e-14, max_iter=5000, precond=kind, smoother=sm,
                              raise_on=(1, 2, 6))
        wref = w.clone()
        st, inf = rr.rr_solve(R.h, lam, y, w, tol=1e-300, x_ref=wref, err_tol=1e-10,
                              max_iter=5000, precond=kind, smoother=sm, raise_on=(1, 2, 6))
        k = inf["iters"]
        torch.cuda.synchronize()
        ta = time.perf_counter()
        rr.rr_solve(R.h, lam, y, w, fixed_iters=k, precond=kind, smoother=sm, chunk=16,
                    raise_on=(1, 2, 6))
        torch.cuda.synchronize()
        compare[name] = {"lambda": lam, "iters": k, "ms": (time.perf_counter() - ta) * 1e3}
    compare["vcycle"] = {"lambda": 1.0, "iters": calib[1.0]["iters"], "ms": last[1.0]["ms"]}
    # flexible CG (truncation 1) with the same V(1,1) preconditioner
    lam = 1.0
    st, inf = rr.rr_solve(R.h, lam, y, w, tol=1e-14, max_iter=5000, precond="vcycle", krylov="fcg",
                          fcg_m=1, raise_on=(1, 2, 6))
    wref = w.clone()
    st, inf = rr.rr_solve(R.h, lam, y, w, tol=1e-300, x_ref=wref, err_tol=1e-10, max_iter=5000,
                          precond="vcycle", krylov="fcg", fcg_m=1, raise_on=(1, 2, 6))
    k = inf["iters"]
    torch.cuda.synchronize()
    ta = time.perf_counter()
    rr.rr_solve(R.h, lam, y, w, fixed_iters=k, precond="vcycle", krylov="fcg", fcg_m=1, chunk=16,
                raise_on=(1, 2, 6))
    torch.cuda.synchronize()
    compare["fcg1_vcycle"] = {"lambda": lam, "iters": k, "ms": (time.perf_counter() - ta) * 1e3}
    # the paper's configuration (TLFCG): flexible CG, two CG steps as rougher;
    # and the variant whose rougher steps are Jacobi-preconditioned
    for name, jac in (("tlfcg", False), ("tlfcg_jacobi_rougher", True)):
        st, inf = rr.rr_solve(R.h, lam, y, w, tol=1e-14, max_iter=5000, precond="rougher",
                              krylov="fcg", fcg_m=1, rougher_jacobi=jac, raise_on=(1, 2, 6))
        wref = w.clone()
        st, inf = rr.rr_solve(R.h, lam, y, w, tol=1e-300, x_ref=wref, err_tol=1e-10, max_iter=5000,
                              precond="rougher", krylov="fcg", fcg_m=1, rougher_jacobi=jac,
                              raise_on=(1, 2, 6))
        k = inf["iters"]
        torch.cuda.synchronize()
        ta = time.perf_counter()
        rr.rr_solve(R.h, lam, y, w, fixed_iters=k, precond="rougher", krylov="fcg", fcg_m=1,
                    rougher_jacobi=jac, chunk=16, raise_on=(1, 2, 6))
        torch.cuda.synchronize()
        compare[name] = {"lambda": lam, "iters": k, "ms": (time.perf_counter() - ta) * 1e3}

    # batched form: the three lambdas as one rr_solve_batched call on the same
    # handle (three work sets, concurrent) against three rr_solve calls, both
    # stopping at relative residual 1e-10
    def seq_solves():
        out = []
        for lam in lams:
            st, inf = rr.rr_solve(R.h, lam, y, w, tol=1e-10, precond="vcycle", chunk=16,
                                  raise_on=(1, 2, 6))
            out.append(inf["iters"])
        return out
    wsb = [torch.empty(F, dtype=torch.float64, device=dev) for _ in lams]
    def batched_solves():
        st, infos = rr.rr_solve_batched([R.h] * len(lams), lams, [y] * len(lams), wsb, tol=1e-10,
                                        precond="vcycle", chunk=16, raise_on=(1, 2, 6))
        return [i["iters"] for i in infos]
    batched = {}
    for name, f in (("plain", seq_solves), ("batched", batched_solves)):
        f()
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for _ in range(3):
            its = f()
        torch.cuda.synchronize()
        batched[name + "_ms"] = (time.perf_counter() - ta) * 1e3 / 3
        batched[name + "_iters"] = its
    batched["speedup"] = batched["plain_ms"] / batched["batched_ms"]

    # mixed precision: FP64 flexible CG (one direction kept) whose V(1,1)
    # cycle runs in FP32, each lambda run for the iterations that reach
    # relative error 1e-10 against the reference (calibrated as for the plain
    # step), against the plain step; the refinement form (FP32 inner PCG
    # restarted at every refinement step) is timed once beside it
    mixed = {"form": "f32_cycle: FP64 FCG(1), Krylov space and operator FP64, V(1,1) cycle in FP32",
             "per_lambda": {}}
    mk = dict(precond="vcycle", krylov="fcg", fcg_m=1, precision="f32_cycle")
    for lam in lams:
        st, inf = rr.rr_solve(R.h, lam, y, w, tol=1e-300, x_ref=wrefs[lam], err_tol=1e-10,
                              max_iter=3000, raise_on=(1, 2, 6), **mk)
        mixed["per_lambda"][str(lam)] = {"iters": inf["iters"], "err": inf["err"]}
    def mixed_step():
        for lam in lams:
            rr.rr_solve(R.h, lam, y, w, fixed_iters=mixed["per_lambda"][str(lam)]["iters"], chunk=16,
                        raise_on=(1, 2, 6), **mk)
    mixed_step()
    torch.cuda.synchronize()
    ta = time.perf_counter()
    for _ in range(3):
        mixed_step()
    torch.cuda.synchronize()
    mixed["ms_per_step"] = (time.perf_counter() - ta) * 1e3 / 3
    mixed["vs_plain"] = ms_per_step / mixed["ms_per_step"]
    ir = {}
    for lam in lams:
        for otol in (1e-10, 3e-11, 1e-11, 3e-12, 1e-12, 3e-13, 1e-13):
            st, inf = rr.rr_solve(R.h, lam, y, w, tol=otol, max_iter=3000, precond="vcycle",
                                  precision="f32_ir", chunk=16, raise_on=(1, 2, 6))
            err = float(torch.linalg.norm(w - wrefs[lam]) / torch.linalg.norm(wrefs[lam]))
            if err <= 1e-10:
                break
        ir[str(lam)] = {"outer_tol": otol, "err": err, "ir_steps": inf["ir_steps"],
                        "inner_iters": inf["iters"], "ms": inf["ms"]}
    mixed["refinement"] = {"per_lambda": ir, "ms_per_step": sum(v["ms"] for v in ir.values())}
    log(f"[bench mixed] FP32 cycle: {mixed['ms_per_step']:.1f} ms per step ({mixed['vs_plain']:.2f}x "
        f"the FP64 step); refinement {mixed['refinement']['ms_per_step']:.1f} ms")

    # learned coarse correction: about 10,000 pairs from V(1,1) solves at
    # lambda log-uniform in [1e-2, 100], Adam on the BF16 network, then
    # flexible CG with the network against V(1,1) PCG at lambda = 1, both to
    # relative residual 1e-10
    learned = {}
    fc = sinfo["n_coarse"]
    llams = list(np.exp(np.random.default_rng(2).uniform(np.log(1e-2), np.log(100.0), 250)))
    per = 40
    inp = torch.empty((len(llams) * per, fc + 1), dtype=torch.float32, device=dev)
    tgt = torch.empty((len(llams) * per, fc), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    npairs = rr.rr_collect_pairs(R.h, llams, per, 1, y, inp, tgt)
    torch.cuda.synchronize()
    learned["collect_s"] = time.perf_counter() - ta
    rr.rr_mlp_init(R.h, hidden=256, seed=11)
    ta = time.perf_counter()
    hist = rr.rr_mlp_train(R.h, inp[:npairs].contiguous(), tgt[:npairs].contiguous(), epochs=60,
                           batch=256, lr=1e-3, seed=5)
    torch.cuda.synchronize()
    learned.update({"pairs": npairs, "train_s": time.perf_counter() - ta, "epochs": 60,
                    "loss_first": hist[0], "loss_last": hist[-1]})
    # the fit: the network's relative error on its own training pairs (the
    # targets are the coarse corrections in units of the coarse Jacobi step)
    outp = torch.empty_like(tgt[:npairs])
    rr.rr_mlp_forward(R.h, inp[:npairs].contiguous(), outp)
    Tt = tgt[:npairs].double()
    rel = (torch.linalg.norm(outp.double() - Tt, dim=1) / torch.linalg.norm(Tt, dim=1)).cpu().numpy()
    learned["fit_relative_error"] = {"median": float(np.median(rel)), "p90": float(np.quantile(rel, 0.9))}
    def learned_solve():
        kw = dict(precond="learned", krylov="fcg", fcg_m=4)
        st, inf = rr.rr_solve(R.h, 1.0, y, w, tol=1e-10, max_iter=5000, chunk=8, raise_on=(1, 2, 6), **kw)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        st, inf = rr.rr_solve(R.h, 1.0, y, w, tol=1e-10, max_iter=5000, chunk=8, raise_on=(1, 2, 6), **kw)
        torch.cuda.synchronize()
        return {"iters": inf["iters"], "ms": (time.perf_counter() - ta) * 1e3,
                "true_relres": inf["true_relres"], "fallback_iter": inf["fallback_iter"]}
    learned["learned_fcg"] = learned_solve()
    # a second round on-policy: pairs from the network's own solves (the
    # residual directions a solve it steers produces), 20 more epochs on the
    # union of both sets
    llams2 = llams[:100]
    inp2 = torch.empty((len(llams2) * per, fc + 1), dtype=torch.float32, device=dev)
    tgt2 = torch.empty((len(llams2) * per, fc), dtype=torch.float32, device=dev)
    n2 = rr.rr_collect_pairs_learned(R.h, llams2, per, 1, y, inp2, tgt2)
    hist2 = rr.rr_mlp_train(R.h, torch.cat([inp[:npairs], inp2[:n2]]).contiguous(),
                            torch.cat([tgt[:npairs], tgt2[:n2]]).contiguous(), epochs=20, batch=256,
                            lr=5e-4, seed=6)
    learned["on_policy_pairs"] = n2
    learned["on_policy_loss_last"] = hist2[-1]
    learned["learned_fcg_on_policy"] = learned_solve()
    for name, kw in (("vcycle_pcg", dict(precond="vcycle")),
                     ("jacobi_fcg", dict(precond="jacobi", krylov="fcg", fcg_m=4))):
        st, inf = rr.rr_solve(R.h, 1.0, y, w, tol=1e-10, max_iter=5000, chunk=8, raise_on=(1, 2, 6), **kw)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        st, inf = rr.rr_solve(R.h, 1.0, y, w, tol=1e-10, max_iter=5000, chunk=8, raise_on=(1, 2, 6), **kw)
        torch.cuda.synchronize()
        learned[name] = {"iters": inf["iters"], "ms": (time.perf_counter() - ta) * 1e3,
                         "true_relres": inf["true_relres"], "fallback_iter": inf["fallback_iter"]}

    total_iters = sum(calib[l]["iters"] for l in lams)
    cpu = None
    if orc is not None:
        cpu_s = sum(orc[l]["s_per_iter"] * calib[l]["iters"] for l in lams)
        cores = len(os.sched_getaffinity(0))
        cpu = {"value": cpu_s, "unit": "s", "cores": 1, "kind": "oracle",
               "sample": "the oracle's three reference solves (V(1,1) two-level PCG on the GPU's "
                         "k-means aggregation, lambda in {1e-2, 1, 100}, to relative residual 1e-13: "
                         + ", ".join(f"{orc[l]['iters']} iterations in {orc[l]['s']:.1f} s" for l in lams)
                         + f") on one thread (SciPy sparse products are single-threaded and BLAS is "
                           f"held to one thread; {cores} cores visible); seconds per iteration of "
                           f"each lambda times the step's iteration count for it"}

    bayes = None if args.no_dense else bayes_section(rr, torch, dev, log, P, R, args.k)
    newton = None if args.no_dense else newton_section(rr, torch, dev, log, P, args.k)
    lf = None if args.no_dense else leader_section(rr, torch, dev, log, P, R)
    tiny = None if args.no_dense else tiny_section(rr, torch, dev, log)
    dense = None if args.no_dense else dense_section(rr, torch, dev, log)
    uneven = None if args.no_dense else batched_uneven_section(rr, torch, dev, log,
                                                               full=not args.batched_small)

    line = {
        "metric": METRIC,
        "value": ms_per_step / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Zipf(1.1) binary fingerprints, y = X w* + N(0, 0.1^2))",
        "config": {
            "workload": "binary 200000x100000 CSR+CSC, 60 nnz/row (12.0M nnz), Zipf(1.1) columns; "
                        "k-means k=1000 feature aggregation; V(1,1) two-level PCG (damped Jacobi "
                        "smoothing, FP64 coarse Cholesky); lambda in {1e-2,1,100}; each solve run "
                        "to relative error <= 1e-10 vs a converged reference",
            "lambdas": lams,
            "n_clusters": args.k,
            "n_coarse": sinfo["n_coarse"],
        },
        "reference": "oracle" if orc is not None else "gpu",
        "per_lambda": {str(l): {"iters": last[l]["iters"], "ms": last[l]["ms"],
                                "err": calib[l]["err"],
                                "err_final": err_final[l],
                                "coarse_factor_ms": calib[l]["coarse_ms"],
                                "oracle_iters_to_relres_1e-10": calib[l].get("oracle_iters_to_relres_1e-10"),
                                "gpu_iters_to_relres_1e-10": calib[l].get("gpu_iters_to_relres_1e-10")}
                       for l in lams},
        "setup_ms": sinfo["setup_ms"],
        "autotune": {"plan_ms": sinfo["plan_ms"], "rows_div": sinfo["tuned_rows_div"],
                     "cols_div": sinfo["tuned_cols_div"], "cached": sinfo["tune_cached"]},
        "kmeans_ms": sinfo["kmeans_ms"],
        "kmeans_passes": sinfo["kmeans_iters"],
        "operator": {"apply_bytes": b_apply, "apply_ms": apply_ms, "apply_gbs": gbs_op,
                     "row_pass_ms": gcsr_ms, "column_pass_ms": col_ms, "column_gather_ms": gcsc_ms,
                     "in_solve_row_pass_ms": csr_ms, "in_solve_column_pass_ms": csc_ms},
        "compare_lambda1": compare,
        "batched_lambdas": batched,
        "mixed_precision": mixed,
        "learned": learned,
        "dense_many_rhs": dense,
        "batched_uneven": uneven,
        "bayes_noise_injection": bayes,
        "newton_logistic": newton,
        "leader_follower": lf,
        "tiny_plain": tiny,
        "operator_valued_f64": valued,
        "roofline": {"bound": "hbm", "achieved": gbs_op, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs_op / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel": "one operator application q = X^T (X p) + lambda p (rr::k_rows row "
                               "pass, rr::k_sell<1> column gather, rr::k_sell_reduce<2> column sums "
                               "and epilogue), HIP events on the solve's stream around 20 "
                               "back-to-back launches of the row pass and of the column pass on "
                               "each timed solve's final vectors",
                     "bytes_per_launch": b_apply, "ms_per_launch": apply_ms,
                     "cache_resident": "the pattern's index arrays and vectors (about 60 MB) stay in "
                                       "the 256 MB Infinity Cache between passes; operator_valued_f64 "
                                       "is the HBM-resident case",
                     "column_gather": {"kernel": "rr::k_sell<1>", "bytes": b_gather, "ms": gcsc_ms,
                                       "gbs": gbs_gather, "frac": gbs_gather / HBM_PEAK_GBS}},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    if args.calibrate_copy:
        calibration_copy(torch, dev)


def calibration_copy(torch, dev):
    """A plain 256 MiB device-to-device copy: what FETCH_SIZE and WRITE_SIZE
    read for it scales the counters to bytes."""
    a = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()


if __name__ == "__main__":
    main()
