"""MI355X two-level preconditioned CG for ridge regression.

A thin ctypes binding over ``librr.so``, the HIP/CDNA4 library whose C ABI
is ``include/rr.h``.  The functions below carry the ABI's names and only
marshal arguments: PyTorch supplies device memory (tensors on ``cuda``) and
the stream (``torch.cuda.current_stream()``); every step of the solver runs
in the library's kernels.  If the library is not built, importing this
package raises ImportError.

Method: Tavernier, Simm, Meerbergen & Moreau, "Two-level preconditioning for
Ridge Regression" (arXiv 1806.05826): (X^T X + lambda I) w = X^T y solved by
PCG with a two-level preconditioner whose coarse space aggregates feature
columns by k-means++ (the paper's beta is lambda here).
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librr.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is not built; run `python -c 'import __graft_entry__ as g; g.build()'` "
        "or `python paper_1806_05826_amd/build.py`")

_lib = C.CDLL(LIB_PATH)

RR_OK, RR_ERR_INVALID_ARG, RR_ERR_DEVICE, RR_ERR_WORKSPACE = 0, 1, 2, 3
RR_ERR_NOT_CONVERGED, RR_ERR_BREAKDOWN, RR_ERR_UNSUPPORTED = 4, 5, 6
PRECOND = {"none": 0, "jacobi": 1, "vcycle": 2, "additive": 3, "learned": 4, "rougher": 5}
KRYLOV = {"pcg": 0, "fcg": 1}
SMOOTHER = {"point": 0, "block": 1}
PRECISION = {"f64": 0, "f32_ir": 1, "bf16_ir": 2, "f32_cycle": 3}


class rr_csr(C.Structure):
    _fields_ = [("n_rows", C.c_int64), ("n_cols", C.c_int64), ("nnz", C.c_int64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("values", C.c_void_p)]


class rr_dense(C.Structure):
    _fields_ = [("n_rows", C.c_int64), ("n_cols", C.c_int64), ("ld", C.c_int64),
                ("values", C.c_void_p)]


class _Versioned(C.Structure):
    """An options struct whose first field, struct_size, is set to the
    struct's size on construction (the library reads that many bytes)."""

    def __init__(self, **kw):
        super().__init__(**kw)
        self.struct_size = C.sizeof(self)


class rr_setup_opts(_Versioned):
    _fields_ = [("struct_size", C.c_uint32), ("n_clusters", C.c_int32), ("kmeans_max_iter", C.c_int32),
                ("seed", C.c_uint64), ("labels_in", C.c_void_p), ("n_labels_in", C.c_int32),
                ("lambda_slots", C.c_int32), ("autotune", C.c_int32),
                ("block_smoother", C.c_int32), ("coarse_eigen", C.c_int32),
                ("lf_tolerance", C.c_double), ("reserve_fcg_m", C.c_int32),
                ("reserve_sets", C.c_int32), ("reserve_f32", C.c_int32), ("reserved0", C.c_int32)]


class rr_setup_info(C.Structure):
    _fields_ = [("n_rows", C.c_int64), ("n_cols", C.c_int64), ("nnz", C.c_int64),
                ("n_coarse", C.c_int32), ("n_centres", C.c_int32), ("kmeans_iters", C.c_int32),
                ("binary", C.c_int32), ("setup_ms", C.c_double), ("kmeans_ms", C.c_double),
                ("plan_ms", C.c_double), ("tuned_rows_div", C.c_int32),
                ("tuned_cols_div", C.c_int32), ("tune_cached", C.c_int32), ("dense", C.c_int32),
                ("dense_split", C.c_int32 * 3), ("dense_split_cached", C.c_int32),
                ("eigen_sweeps", C.c_int32)]


class rr_solve_opts(_Versioned):
    _fields_ = [("struct_size", C.c_uint32), ("reserved0", C.c_int32), ("tol", C.c_double), ("max_iter", C.c_int32), ("fixed_iters", C.c_int32),
                ("precond", C.c_int32), ("rhs_is_b", C.c_int32), ("omega", C.c_double),
                ("x_ref", C.c_void_p), ("err_tol", C.c_double),
                ("residual_history", C.c_void_p), ("chunk", C.c_int32), ("profile", C.c_int32),
                ("krylov", C.c_int32), ("fcg_m", C.c_int32), ("precision", C.c_int32),
                ("graph", C.c_int32), ("inner_tol", C.c_double), ("smoother", C.c_int32),
                ("rougher_steps", C.c_int32), ("rougher_jacobi", C.c_int32),
                ("persistent", C.c_int32), ("hybrid_iters", C.c_int32)]


class rr_solve_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("op_applies", C.c_int32),
                ("ir_steps", C.c_int32), ("relres", C.c_double), ("true_relres", C.c_double),
                ("err", C.c_double), ("omega", C.c_double), ("ms", C.c_double),
                ("coarse_ms", C.c_double), ("csr_avg_ms", C.c_double),
                ("csc_avg_ms", C.c_double), ("csr_launches", C.c_int32),
                ("csc_launches", C.c_int32), ("csr_gather_avg_ms", C.c_double),
                ("csc_gather_avg_ms", C.c_double), ("fallback_iter", C.c_int32),
                ("pad_", C.c_int32)]


_P = C.c_void_p
_SIGS = {
    "rr_setup": [C.POINTER(rr_csr), C.POINTER(rr_setup_opts), _P, C.POINTER(_P)],
    "rr_destroy": [_P],
    "rr_get_setup_info": [_P, C.POINTER(rr_setup_info)],
    "rr_get_labels": [_P, _P, _P],
    "rr_get_centres": [_P, _P, _P],
    "rr_solve": [_P, C.c_double, _P, _P, C.POINTER(rr_solve_opts), C.POINTER(rr_solve_info), _P],
    "rr_solve_batched": [C.c_int32, _P, _P, _P, _P, C.POINTER(rr_solve_opts), _P, _P],
    "rr_mlp_init": [_P, C.c_int32, C.c_uint64],
    "rr_mlp_size": [_P, _P, _P, _P],
    "rr_mlp_set_weights": [_P, _P],
    "rr_mlp_get_weights": [_P, _P],
    "rr_mlp_forward": [_P, _P, C.c_int32, _P, _P],
    "rr_mlp_backward": [_P, _P, _P, C.c_int32, _P, _P],
    "rr_mlp_train": [_P, _P, _P, C.c_int64, _P, _P, _P],
    "rr_collect_pairs": [_P, _P, C.c_int32, C.c_int32, C.c_int32, _P, _P, _P, _P, _P],
    "rr_collect_pairs_learned": [_P, _P, C.c_int32, C.c_int32, C.c_int32, _P, _P, _P, _P, _P],
    "rr_apply_operator": [_P, C.c_double, _P, _P, _P],
    "rr_apply_rhs": [_P, _P, _P, _P],
    "rr_apply_precond": [_P, C.c_double, C.c_int32, C.c_double, _P, _P, _P],
    "rr_coarse_gram": [_P, _P, _P],
    "rr_coarse_factor": [_P, C.c_double, _P, _P, _P],
    "rr_coarse_eigen": [_P, _P, _P, _P],
    "rr_noise_rhs": [_P, C.c_double, C.c_double, _P, _P, _P, _P, _P],
    "rr_set_row_weights": [_P, _P, _P],
    "rr_apply_rows": [_P, _P, _P, _P],
    "rr_set_interpolation": [_P, _P, C.c_int32, C.c_double, _P, _P, _P],
    "rr_smoother_weight": [_P, C.c_double, C.POINTER(C.c_double)],
    "rr_setup_dense": [C.POINTER(rr_dense), C.POINTER(rr_setup_opts), _P, C.POINTER(_P)],
    "rr_solve_block": [_P, C.c_double, C.c_int32, _P, C.c_int64, _P, C.c_int64,
                       C.POINTER(rr_solve_opts), _P, _P],
    "rr_apply_operator_block": [_P, C.c_double, C.c_int32, _P, C.c_int64, _P, C.c_int64,
                                C.c_int32, _P],
    "rr_setup_ws": [C.POINTER(rr_csr), C.POINTER(rr_setup_opts), _P, C.c_size_t, _P, C.POINTER(_P)],
    "rr_setup_workspace_size": [C.POINTER(rr_csr), C.POINTER(rr_setup_opts), _P,
                                C.POINTER(C.c_size_t)],
    "rr_set_allocator": [_P, _P, _P],
    "rr_prototypes": [_P, C.c_int32, C.c_int32, C.c_uint64, _P, _P, _P],
    "rr_solve_batched_noalloc": [C.c_int32, _P, _P, _P, _P, C.POINTER(rr_solve_opts), _P, _P],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int
_lib.rr_last_error.argtypes = []
_lib.rr_last_error.restype = C.c_char_p


# --- device memory: PyTorch's caching allocator supplies the library's memory

_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_int32, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_int32, C.c_void_p)


def _torch_alloc(nbytes, device, ctx):
    try:
        import torch
        return torch.cuda.caching_allocator_alloc(int(nbytes), device=int(device))
    except Exception:   # the library reports the failed allocation
        return None


def _torch_free(ptr, device, ctx):
    try:
        import torch
        torch.cuda.caching_allocator_delete(int(ptr))
    except Exception:   # interpreter shutdown: torch may already be gone
        pass


_torch_alloc_c = _ALLOC_FN(_torch_alloc)
_torch_free_c = _FREE_FN(_torch_free)


def rr_set_allocator(use_torch=True):
    """Route the device memory of handles set up from now on through
    PyTorch's caching allocator (the default at import), or back to
    hipMalloc with use_torch=False."""
    if use_torch:
        _check(_lib.rr_set_allocator(C.cast(_torch_alloc_c, C.c_void_p),
                                     C.cast(_torch_free_c, C.c_void_p), None))
    else:
        _check(_lib.rr_set_allocator(None, None, None))


class RRError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"rr status {status}: {message}")
        self.status = status
        self.message = message


def rr_last_error() -> str:
    return (_lib.rr_last_error() or b"").decode()


def _check(st: int, allow=()):
    if st != RR_OK and st not in allow:
        raise RRError(st, rr_last_error())
    return st


if os.environ.get("RR_TORCH_ALLOCATOR", "1") != "0":
    rr_set_allocator(True)


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev_f64(t, n=None, name="vector"):
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise ValueError(f"{name}: need a contiguous float64 CUDA tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name}: expected {n} elements, got {t.numel()}")
    return t


# --- the C ABI, one Python function per entry point -------------------------

def _setup_args(row_ptr, col_idx, values, n_cols, n_clusters=0, seed=0, kmeans_max_iter=0,
                labels_in=None, n_labels_in=0, lambda_slots=0, autotune=False, block_smoother=False,
                coarse_eigen=False, lf_tolerance=0.0, reserve_fcg_m=0, reserve_sets=0,
                reserve_f32=False):
    import torch
    for t, nm in ((row_ptr, "row_ptr"), (col_idx, "col_idx")):
        if not (t.is_cuda and t.dtype == torch.int32 and t.is_contiguous()):
            raise ValueError(f"{nm}: need a contiguous int32 CUDA tensor")
    if values is not None:
        _dev_f64(values, col_idx.numel(), "values")
    if labels_in is not None and not (labels_in.is_cuda and labels_in.dtype == torch.int32):
        raise ValueError("labels_in: need an int32 CUDA tensor")
    X = rr_csr(row_ptr.numel() - 1, int(n_cols), col_idx.numel(), _ptr(row_ptr), _ptr(col_idx),
               _ptr(values))
    o = rr_setup_opts(n_clusters=int(n_clusters), kmeans_max_iter=int(kmeans_max_iter),
                      seed=int(seed) & (2**64 - 1), labels_in=_ptr(labels_in),
                      n_labels_in=int(n_labels_in), lambda_slots=int(lambda_slots),
                      autotune=1 if autotune else 0, block_smoother=1 if block_smoother else 0,
                      coarse_eigen=1 if coarse_eigen else 0, lf_tolerance=float(lf_tolerance),
                      reserve_fcg_m=int(reserve_fcg_m), reserve_sets=int(reserve_sets),
                      reserve_f32=1 if reserve_f32 else 0)
    return X, o


def rr_setup(row_ptr, col_idx, values, n_cols, n_clusters=0, seed=0, kmeans_max_iter=0,
             labels_in=None, n_labels_in=0, lambda_slots=0, autotune=False, block_smoother=False,
             coarse_eigen=False, lf_tolerance=0.0, reserve_fcg_m=0, reserve_sets=0,
             reserve_f32=False, workspace=None, stream=None):
    """X is a device CSR: row_ptr/col_idx int32 CUDA tensors, values float64
    CUDA tensor or None (binary).  With ``workspace`` (a contiguous CUDA
    tensor of at least rr_setup_workspace_size bytes, 256-byte aligned) the
    handle lives in that memory (rr_setup_ws).  Returns an opaque handle."""
    import torch
    for t, nm in ((row_ptr, "row_ptr"), (col_idx, "col_idx")):
        if not (t.is_cuda and t.dtype == torch.int32 and t.is_contiguous()):
            raise ValueError(f"{nm}: need a contiguous int32 CUDA tensor")
    if values is not None:
        _dev_f64(values, col_idx.numel(), "values")
    if labels_in is not None and not (labels_in.is_cuda and labels_in.dtype == torch.int32):
        raise ValueError("labels_in: need an int32 CUDA tensor")
    X = rr_csr(row_ptr.numel() - 1, int(n_cols), col_idx.numel(), _ptr(row_ptr), _ptr(col_idx),
               _ptr(values))
    o = rr_setup_opts(n_clusters=int(n_clusters), kmeans_max_iter=int(kmeans_max_iter),
                      seed=int(seed) & (2**64 - 1), labels_in=_ptr(labels_in),
                      n_labels_in=int(n_labels_in), lambda_slots=int(lambda_slots),
                      autotune=1 if autotune else 0, block_smoother=1 if block_smoother else 0,
                      coarse_eigen=1 if coarse_eigen else 0, lf_tolerance=float(lf_tolerance),
                      reserve_fcg_m=int(reserve_fcg_m), reserve_sets=int(reserve_sets),
                      reserve_f32=1 if reserve_f32 else 0)
    h = C.c_void_p()
    if workspace is None:
        _check(_lib.rr_setup(C.byref(X), C.byref(o), _stream(stream), C.byref(h)))
    else:
        if not (workspace.is_cuda and workspace.is_contiguous()):
            raise ValueError("workspace: need a contiguous CUDA tensor")
        nbytes = workspace.numel() * workspace.element_size()
        _check(_lib.rr_setup_ws(C.byref(X), C.byref(o), _ptr(workspace), C.c_size_t(nbytes),
                                _stream(stream), C.byref(h)))
    return h.value


def rr_setup_ws(row_ptr, col_idx, values, n_cols, workspace, stream=None, **opts):
    """rr_setup with the handle's device memory carved out of ``workspace``
    (a contiguous CUDA tensor of at least rr_setup_workspace_size bytes)."""
    return rr_setup(row_ptr, col_idx, values, n_cols, workspace=workspace, stream=stream, **opts)


def rr_setup_workspace_size(row_ptr, col_idx, values, n_cols, stream=None, **opts):
    """Bytes of device workspace rr_setup_ws needs for this X and options
    (the same keyword options as rr_setup; runs one setup to measure)."""
    X, o = _setup_args(row_ptr, col_idx, values, n_cols, **opts)
    n = C.c_size_t()
    _check(_lib.rr_setup_workspace_size(C.byref(X), C.byref(o), _stream(stream), C.byref(n)))
    return n.value


def _rows_f64(t, name):
    """A (count, n) float64 CUDA tensor whose rows are the block's columns."""
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.dim() == 2 and t.stride(1) == 1):
        raise ValueError(f"{name}: need a 2-D float64 CUDA tensor with unit column stride")
    return t


def rr_setup_dense(X, n_clusters=0, seed=0, kmeans_max_iter=0, labels_in=None, n_labels_in=0,
                   lambda_slots=0, autotune=False, coarse_eigen=False, stream=None):
    """X: (N, F) float32 CUDA tensor with unit column stride (row-major).
    Returns an opaque handle (int)."""
    import torch
    if not (X.is_cuda and X.dtype == torch.float32 and X.dim() == 2 and X.stride(1) == 1):
        raise ValueError("X: need a 2-D float32 CUDA tensor with unit column stride")
    if labels_in is not None and not (labels_in.is_cuda and labels_in.dtype == torch.int32):
        raise ValueError("labels_in: need an int32 CUDA tensor")
    D = rr_dense(X.shape[0], X.shape[1], X.stride(0), _ptr(X))
    o = rr_setup_opts(n_clusters=int(n_clusters), kmeans_max_iter=int(kmeans_max_iter),
                      seed=int(seed) & (2**64 - 1), labels_in=_ptr(labels_in),
                      n_labels_in=int(n_labels_in), lambda_slots=int(lambda_slots),
                      autotune=1 if autotune else 0, coarse_eigen=1 if coarse_eigen else 0)
    h = C.c_void_p()
    _check(_lib.rr_setup_dense(C.byref(D), C.byref(o), _stream(stream), C.byref(h)))
    return h.value


def rr_solve_block(h, lam, rhs, w, tol=0.0, max_iter=0, fixed_iters=0, precond="vcycle",
                   rhs_is_b=False, omega=0.0, precision="f64", inner_tol=0.0, stream=None,
                   raise_on=(RR_ERR_INVALID_ARG, RR_ERR_DEVICE, RR_ERR_UNSUPPORTED)):
    """rhs: (m, N) (or (m, F) with rhs_is_b), w: (m, F); row c is column c
    of the block.  Returns (status, [info dict per column])."""
    _rows_f64(rhs, "rhs")
    _rows_f64(w, "w")
    m = rhs.shape[0]
    if w.shape[0] != m:
        raise ValueError("rhs and w need the same number of rows")
    o = rr_solve_opts(tol=float(tol), max_iter=int(max_iter), fixed_iters=int(fixed_iters),
                      precond=PRECOND[precond] if isinstance(precond, str) else int(precond),
                      rhs_is_b=1 if rhs_is_b else 0, omega=float(omega),
                      precision=PRECISION[precision] if isinstance(precision, str) else int(precision),
                      inner_tol=float(inner_tol))
    infos = (rr_solve_info * max(m, 1))()
    st = _lib.rr_solve_block(C.c_void_p(h), float(lam), int(m), _ptr(rhs), C.c_int64(rhs.stride(0)),
                             _ptr(w), C.c_int64(w.stride(0)), C.byref(o), C.cast(infos, C.c_void_p),
                             _stream(stream))
    if st in raise_on:
        raise RRError(st, rr_last_error())
    return st, [{f: getattr(infos[i], f) for f, _ in rr_solve_info._fields_} for i in range(m)]


def rr_apply_operator_block(h, lam, v, q, precision="f64", stream=None):
    """q[c] = (X^T X + lam I) v[c] for the rows of v (m, F); q (m, F)."""
    _rows_f64(v, "v")
    _rows_f64(q, "q")
    if v.shape != q.shape:
        raise ValueError("v and q need the same shape")
    _check(_lib.rr_apply_operator_block(
        C.c_void_p(h), float(lam), int(v.shape[0]), _ptr(v), C.c_int64(v.stride(0)), _ptr(q),
        C.c_int64(q.stride(0)), PRECISION[precision] if isinstance(precision, str) else int(precision),
        _stream(stream)))


def rr_destroy(h):
    _check(_lib.rr_destroy(C.c_void_p(h)))


def rr_get_setup_info(h) -> dict:
    i = rr_setup_info()
    _check(_lib.rr_get_setup_info(C.c_void_p(h), C.byref(i)))
    out = {}
    for f, _ in rr_setup_info._fields_:
        v = getattr(i, f)
        out[f] = list(v) if isinstance(v, C.Array) else v
    return out


def rr_get_labels(h, labels, stream=None):
    _check(_lib.rr_get_labels(C.c_void_p(h), _ptr(labels), _stream(stream)))


def rr_get_centres(h, centres, stream=None):
    _check(_lib.rr_get_centres(C.c_void_p(h), _ptr(centres), _stream(stream)))


def rr_solve(h, lam, rhs, w, tol=0.0, max_iter=0, fixed_iters=0, precond="vcycle",
             rhs_is_b=False, omega=0.0, x_ref=None, err_tol=0.0, residual_history=None,
             chunk=0, profile=False, krylov="pcg", fcg_m=0, precision="f64", inner_tol=0.0,
             graph=False, smoother="point", rougher_steps=0, rougher_jacobi=False, stream=None,
             raise_on=(RR_ERR_INVALID_ARG, RR_ERR_DEVICE, RR_ERR_UNSUPPORTED)):
    """Returns (status, info dict).  Statuses in `raise_on` raise RRError."""
    _dev_f64(rhs, None, "rhs")
    _dev_f64(w, None, "w")
    o = rr_solve_opts(tol=float(tol), max_iter=int(max_iter), fixed_iters=int(fixed_iters),
                      precond=PRECOND[precond] if isinstance(precond, str) else int(precond),
                      rhs_is_b=1 if rhs_is_b else 0, omega=float(omega), x_ref=_ptr(x_ref),
                      err_tol=float(err_tol), residual_history=_ptr(residual_history),
                      chunk=int(chunk), profile=int(profile),
                      krylov=KRYLOV[krylov] if isinstance(krylov, str) else int(krylov),
                      fcg_m=int(fcg_m),
                      precision=PRECISION[precision] if isinstance(precision, str) else int(precision),
                      graph=1 if graph else 0, inner_tol=float(inner_tol),
                      smoother=SMOOTHER[smoother] if isinstance(smoother, str) else int(smoother),
                      rougher_steps=int(rougher_steps), rougher_jacobi=1 if rougher_jacobi else 0)
    info = rr_solve_info()
    st = _lib.rr_solve(C.c_void_p(h), float(lam), _ptr(rhs), _ptr(w), C.byref(o), C.byref(info),
                       _stream(stream))
    if st in raise_on:
        raise RRError(st, rr_last_error())
    return st, {f: getattr(info, f) for f, _ in rr_solve_info._fields_}


def rr_solve_batched(handles, lams, rhs, ws, tol=0.0, max_iter=0, fixed_iters=0, precond="vcycle",
                     rhs_is_b=False, omega=0.0, chunk=0, krylov="pcg", fcg_m=0, smoother="point",
                     graph=False, persistent=False, hybrid_iters=0, stream=None,
                     raise_on=(RR_ERR_INVALID_ARG, RR_ERR_DEVICE, RR_ERR_UNSUPPORTED)):
    """Batched solves; returns (status, [info dict per problem]).  persistent:
    False (work sets on streams), True (one persistent launch) or "hybrid"
    (the launch with per-problem iteration caps, then the streams)."""
    n = len(handles)
    if not (len(lams) == len(rhs) == len(ws) == n):
        raise ValueError("handles, lams, rhs and ws must have equal lengths")
    for t in list(rhs) + list(ws):
        _dev_f64(t, None, "vector")
    H = (C.c_void_p * max(n, 1))(*[C.c_void_p(h) for h in handles])
    L = (C.c_double * max(n, 1))(*[float(x) for x in lams])
    Rp = (C.c_void_p * max(n, 1))(*[_ptr(t) for t in rhs])
    Wp = (C.c_void_p * max(n, 1))(*[_ptr(t) for t in ws])
    o = rr_solve_opts(tol=float(tol), max_iter=int(max_iter), fixed_iters=int(fixed_iters),
                      precond=PRECOND[precond] if isinstance(precond, str) else int(precond),
                      rhs_is_b=1 if rhs_is_b else 0, omega=float(omega), chunk=int(chunk),
                      krylov=KRYLOV[krylov] if isinstance(krylov, str) else int(krylov),
                      fcg_m=int(fcg_m), graph=1 if graph else 0,
                      smoother=SMOOTHER[smoother] if isinstance(smoother, str) else int(smoother),
                      persistent=2 if persistent == "hybrid" else (1 if persistent else 0),
                      hybrid_iters=int(hybrid_iters))
    infos = (rr_solve_info * max(n, 1))()
    st = _lib.rr_solve_batched(C.c_int32(n), C.cast(H, C.c_void_p), C.cast(L, C.c_void_p),
                               C.cast(Rp, C.c_void_p), C.cast(Wp, C.c_void_p), C.byref(o),
                               C.cast(infos, C.c_void_p), _stream(stream))
    if st in raise_on:
        raise RRError(st, rr_last_error())
    return st, [{f: getattr(infos[i], f) for f, _ in rr_solve_info._fields_} for i in range(n)]


def rr_solve_batched_noalloc(handles, lams, rhs, ws, tol=0.0, max_iter=0, fixed_iters=0,
                             precond="vcycle", rhs_is_b=False, omega=0.0, stream=None,
                             raise_on=(RR_ERR_INVALID_ARG, RR_ERR_DEVICE, RR_ERR_WORKSPACE,
                                       RR_ERR_UNSUPPORTED)):
    """The persistent batched solve with no device allocation (the
    library's static scratch); returns (status, [info dict per problem])."""
    n = len(handles)
    if not (len(lams) == len(rhs) == len(ws) == n):
        raise ValueError("handles, lams, rhs and ws must have equal lengths")
    for t in list(rhs) + list(ws):
        _dev_f64(t, None, "vector")
    H = (C.c_void_p * max(n, 1))(*[C.c_void_p(h) for h in handles])
    L = (C.c_double * max(n, 1))(*[float(x) for x in lams])
    Rp = (C.c_void_p * max(n, 1))(*[_ptr(t) for t in rhs])
    Wp = (C.c_void_p * max(n, 1))(*[_ptr(t) for t in ws])
    o = rr_solve_opts(tol=float(tol), max_iter=int(max_iter), fixed_iters=int(fixed_iters),
                      precond=PRECOND[precond] if isinstance(precond, str) else int(precond),
                      rhs_is_b=1 if rhs_is_b else 0, omega=float(omega), persistent=1)
    infos = (rr_solve_info * max(n, 1))()
    st = _lib.rr_solve_batched_noalloc(C.c_int32(n), C.cast(H, C.c_void_p), C.cast(L, C.c_void_p),
                                       C.cast(Rp, C.c_void_p), C.cast(Wp, C.c_void_p), C.byref(o),
                                       C.cast(infos, C.c_void_p), _stream(stream))
    if st in raise_on:
        raise RRError(st, rr_last_error())
    return st, [{f: getattr(infos[i], f) for f, _ in rr_solve_info._fields_} for i in range(n)]


class rr_mlp_train_opts(_Versioned):
    _fields_ = [("struct_size", C.c_uint32), ("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_double),
                ("seed", C.c_uint64)]


def rr_mlp_init(h, hidden=256, seed=0):
    _check(_lib.rr_mlp_init(C.c_void_p(h), int(hidden), C.c_uint64(seed)))


def rr_mlp_size(h):
    n, i, o = C.c_int64(), C.c_int32(), C.c_int32()
    _check(_lib.rr_mlp_size(C.c_void_p(h), C.byref(n), C.byref(i), C.byref(o)))
    return n.value, i.value, o.value


def rr_mlp_set_weights(h, params):
    import numpy as np
    a = np.ascontiguousarray(params, dtype=np.float32)
    _check(_lib.rr_mlp_set_weights(C.c_void_p(h), a.ctypes.data_as(C.c_void_p)))


def rr_mlp_get_weights(h):
    import numpy as np
    n, _, _ = rr_mlp_size(h)
    a = np.empty(n, dtype=np.float32)
    _check(_lib.rr_mlp_get_weights(C.c_void_p(h), a.ctypes.data_as(C.c_void_p)))
    return a


def _dev_f32(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32
            and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float32 CUDA tensor")


def rr_mlp_forward(h, inp, out, stream=None):
    _dev_f32(inp, "in")
    _dev_f32(out, "out")
    _check(_lib.rr_mlp_forward(C.c_void_p(h), _ptr(inp), int(inp.shape[0]), _ptr(out), _stream(stream)))


def rr_mlp_backward(h, inp, dout, grads, stream=None):
    for t, nm in ((inp, "in"), (dout, "dout"), (grads, "grads")):
        _dev_f32(t, nm)
    _check(_lib.rr_mlp_backward(C.c_void_p(h), _ptr(inp), _ptr(dout), int(inp.shape[0]),
                                _ptr(grads), _stream(stream)))


def rr_mlp_train(h, inp, target, epochs=0, batch=0, lr=0.0, seed=0, stream=None):
    """Returns the per-epoch mean loss (host list)."""
    import numpy as np
    _dev_f32(inp, "in")
    _dev_f32(target, "target")
    o = rr_mlp_train_opts(epochs=int(epochs), batch=int(batch), lr=float(lr), seed=int(seed))
    hist = np.zeros(max(1, epochs if epochs > 0 else 20), dtype=np.float32)
    _check(_lib.rr_mlp_train(C.c_void_p(h), _ptr(inp), _ptr(target), C.c_int64(int(inp.shape[0])),
                             C.byref(o), hist.ctypes.data_as(C.c_void_p), _stream(stream)))
    return hist.tolist()


def rr_collect_pairs(h, lams, pairs_per_solve, every, y, inputs, targets, stream=None):
    """Returns the number of pairs written."""
    _dev_f32(inputs, "inputs")
    _dev_f32(targets, "targets")
    _dev_f64(y, None, "y")
    L = (C.c_double * max(1, len(lams)))(*[float(x) for x in lams])
    n = C.c_int64()
    _check(_lib.rr_collect_pairs(C.c_void_p(h), C.cast(L, C.c_void_p), len(lams), int(pairs_per_solve),
                                 int(every), _ptr(y), _ptr(inputs), _ptr(targets), C.byref(n),
                                 _stream(stream)))
    return n.value


def rr_collect_pairs_learned(h, lams, pairs_per_solve, every, y, inputs, targets, stream=None):
    """Pairs from the network's own flexible-CG solves; returns the count."""
    _dev_f32(inputs, "inputs")
    _dev_f32(targets, "targets")
    _dev_f64(y, None, "y")
    L = (C.c_double * max(1, len(lams)))(*[float(x) for x in lams])
    n = C.c_int64()
    _check(_lib.rr_collect_pairs_learned(C.c_void_p(h), C.cast(L, C.c_void_p), len(lams),
                                         int(pairs_per_solve), int(every), _ptr(y), _ptr(inputs),
                                         _ptr(targets), C.byref(n), _stream(stream)))
    return n.value


def rr_apply_operator(h, lam, v, Av, stream=None):
    _check(_lib.rr_apply_operator(C.c_void_p(h), float(lam), _ptr(v), _ptr(Av), _stream(stream)))


def rr_apply_rhs(h, y, b, stream=None):
    _check(_lib.rr_apply_rhs(C.c_void_p(h), _ptr(y), _ptr(b), _stream(stream)))


def rr_noise_rhs(h, tau, lam, y, xi1, xi2, b, stream=None):
    """b = X^T (y + xi1 / sqrt(tau)) + sqrt(lam) / tau * xi2 (device float64)."""
    _check(_lib.rr_noise_rhs(C.c_void_p(h), float(tau), float(lam), _ptr(y), _ptr(xi1), _ptr(xi2),
                             _ptr(b), _stream(stream)))


def rr_set_row_weights(h, d, stream=None):
    """d: float64 CUDA tensor of N weights >= 0, or None to clear them."""
    _check(_lib.rr_set_row_weights(C.c_void_p(h), _ptr(d), _stream(stream)))


def rr_apply_rows(h, v, u, stream=None):
    _check(_lib.rr_apply_rows(C.c_void_p(h), _ptr(v), _ptr(u), _stream(stream)))


def rr_set_interpolation(h, V, n_proto, beta, rep=None, p=None, stream=None):
    """V: float64 CUDA tensor of n_proto * F prototype values (prototype k
    contiguous), or None to restore the adjusted square-root average; rep:
    int32 CUDA tensor of F_C coarse features or None; p: float64 CUDA tensor
    of F receiving the weights, or None."""
    _check(_lib.rr_set_interpolation(C.c_void_p(h), _ptr(V), int(n_proto), float(beta), _ptr(rep),
                                     _ptr(p), _stream(stream)))


def rr_prototypes(h, n_proto, V, steps=0, seed=0x5eed, stream=None):
    """V: (n_proto, F) float64 CUDA tensor receiving the leading
    eigenvectors of X^T X (caller's feature order); returns the Ritz values
    (numpy, descending)."""
    import numpy as np
    _dev_f64(V, None, "V")
    ev = np.empty(int(n_proto), dtype=np.float64)
    _check(_lib.rr_prototypes(C.c_void_p(h), int(n_proto), int(steps), int(seed) & (2**64 - 1),
                              _ptr(V), ev.ctypes.data_as(C.c_void_p), _stream(stream)))
    return ev


def rr_coarse_eigen(h, Q, ev, stream=None):
    _check(_lib.rr_coarse_eigen(C.c_void_p(h), _ptr(Q), _ptr(ev), _stream(stream)))


def rr_apply_precond(h, lam, precond, omega, r, z, stream=None):
    k = PRECOND[precond] if isinstance(precond, str) else int(precond)
    _check(_lib.rr_apply_precond(C.c_void_p(h), float(lam), k, float(omega), _ptr(r), _ptr(z),
                                 _stream(stream)))


def rr_coarse_gram(h, K, stream=None):
    _check(_lib.rr_coarse_gram(C.c_void_p(h), _ptr(K), _stream(stream)))


def rr_coarse_factor(h, lam, L=None, Ainv=None, stream=None):
    _check(_lib.rr_coarse_factor(C.c_void_p(h), float(lam), _ptr(L), _ptr(Ainv), _stream(stream)))


def rr_smoother_weight(h, lam) -> float:
    out = C.c_double()
    _check(_lib.rr_smoother_weight(C.c_void_p(h), float(lam), C.byref(out)))
    return out.value


# --- a small convenience wrapper ---------------------------------------------

class Ridge:
    """Owns one handle.  ``X`` is a scipy CSR matrix (host); it is copied to
    the device, handed to rr_setup and released (the library keeps its own
    copy)."""

    def __init__(self, X, n_clusters=0, seed=0, kmeans_max_iter=0, labels=None, binary=None,
                 lambda_slots=0, autotune=False, block_smoother=False, coarse_eigen=False,
                 lf_tolerance=0.0, reserve_fcg_m=0, reserve_sets=0, reserve_f32=False,
                 workspace=None, device="cuda"):
        import numpy as np
        import torch
        X = X.tocsr()
        X.sort_indices()
        if binary is None:
            binary = bool(X.nnz == 0 or np.all(X.data == 1.0))
        self.N, self.F = X.shape
        self.device = torch.device(device)
        rp = torch.as_tensor(X.indptr.astype(np.int32), device=self.device)
        ci = torch.as_tensor(X.indices.astype(np.int32), device=self.device)
        vals = None if binary else torch.as_tensor(X.data.astype(np.float64), device=self.device)
        lab = None
        nlab = 0
        if labels is not None:
            lab = torch.as_tensor(np.asarray(labels, dtype=np.int32), device=self.device)
            nlab = int(np.max(labels)) + 1 if len(labels) else 1
        self.workspace = workspace   # kept alive with the handle
        self.h = rr_setup(rp, ci, vals, self.F, n_clusters, seed, kmeans_max_iter, lab, nlab,
                          lambda_slots, autotune, block_smoother, coarse_eigen, lf_tolerance,
                          reserve_fcg_m, reserve_sets, reserve_f32, workspace)
        torch.cuda.current_stream().synchronize()
        self.info = rr_get_setup_info(self.h)

    def close(self):
        if getattr(self, "h", None):
            rr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vec(self, v, n):
        import torch
        t = torch.as_tensor(v, dtype=torch.float64, device=self.device).contiguous()
        if t.numel() != n:
            raise ValueError(f"expected {n} elements")
        return t

    def solve(self, lam, y, rhs_is_b=False, **kw):
        import torch
        rhs = self._vec(y, self.F if rhs_is_b else self.N)
        w = torch.empty(self.F, dtype=torch.float64, device=self.device)
        st, info = rr_solve(self.h, lam, rhs, w, rhs_is_b=rhs_is_b, **kw)
        return w, info

    def apply_operator(self, lam, v):
        import torch
        v = self._vec(v, self.F)
        out = torch.empty_like(v)
        rr_apply_operator(self.h, lam, v, out)
        return out

    def apply_rhs(self, y):
        import torch
        y = self._vec(y, self.N)
        out = torch.empty(self.F, dtype=torch.float64, device=self.device)
        rr_apply_rhs(self.h, y, out)
        return out

    def apply_precond(self, lam, r, precond="vcycle", omega=0.0):
        import torch
        r = self._vec(r, self.F)
        z = torch.empty_like(r)
        rr_apply_precond(self.h, lam, precond, omega, r, z)
        return z

    def labels(self):
        import torch
        out = torch.empty(self.F, dtype=torch.int32, device=self.device)
        rr_get_labels(self.h, out)
        return out

    def centres(self):
        import torch
        out = torch.empty(self.info["n_centres"], dtype=torch.int32, device=self.device)
        rr_get_centres(self.h, out)
        return out

    def coarse_gram(self):
        import torch
        fc = self.info["n_coarse"]
        K = torch.empty(fc * fc, dtype=torch.float64, device=self.device)
        rr_coarse_gram(self.h, K)
        return K.view(fc, fc)

    def coarse_factor(self, lam):
        import torch
        fc = self.info["n_coarse"]
        L = torch.empty(fc * fc, dtype=torch.float64, device=self.device)
        Ai = torch.empty_like(L)
        rr_coarse_factor(self.h, lam, L, Ai)
        return L.view(fc, fc), Ai.view(fc, fc)

    def smoother_weight(self, lam):
        return rr_smoother_weight(self.h, lam)

    def coarse_eigen(self):
        """(Q, ev) with K = Q diag(ev) Q^T (a handle set up with coarse_eigen)."""
        import torch
        fc = self.info["n_coarse"]
        Q = torch.empty(fc * fc, dtype=torch.float64, device=self.device)
        ev = torch.empty(fc, dtype=torch.float64, device=self.device)
        rr_coarse_eigen(self.h, Q, ev)
        return Q.view(fc, fc), ev

    def set_row_weights(self, d):
        """The operator becomes X^T D X + lam I (d: N weights >= 0; None clears)."""
        rr_set_row_weights(self.h, None if d is None else self._vec(d, self.N))

    def set_interpolation(self, V, beta=0.0, rep=None):
        """Least-squares interpolation from prototypes V (F x K, or None to
        restore the adjusted square-root average); returns the weights p
        (F) or None."""
        import torch
        if V is None:
            rr_set_interpolation(self.h, None, 0, 0.0)
            return None
        Vt = torch.as_tensor(V, dtype=torch.float64, device=self.device)
        if Vt.dim() != 2 or Vt.shape[0] != self.F:
            raise ValueError("V must be F x K")
        Vk = Vt.t().contiguous()      # prototype k contiguous
        r = None
        if rep is not None:
            fc = self.info["n_coarse"]
            r = torch.as_tensor(rep, device=self.device)
            if r.dtype not in (torch.int32, torch.int64) or r.dim() != 1 or r.numel() != fc:
                raise ValueError(f"rep must be a 1-D integer tensor of n_coarse = {fc} elements")
            r = r.to(torch.int32).contiguous()
        p = torch.empty(self.F, dtype=torch.float64, device=self.device)
        rr_set_interpolation(self.h, Vk, Vt.shape[1], beta, r, p)
        return p

    def apply_rows(self, v):
        import torch
        v = self._vec(v, self.F)
        out = torch.empty(self.N, dtype=torch.float64, device=self.device)
        rr_apply_rows(self.h, v, out)
        return out

    def noise_rhs(self, tau, lam, y, xi1, xi2):
        import torch
        y = self._vec(y, self.N)
        xi1 = self._vec(xi1, self.N)
        xi2 = self._vec(xi2, self.F)
        out = torch.empty(self.F, dtype=torch.float64, device=self.device)
        rr_noise_rhs(self.h, tau, lam, y, xi1, xi2, out)
        return out


class DenseRidge(Ridge):
    """A handle over dense X (N x F, FP32) for blocks of right-hand sides.
    ``X`` is a host array or a CUDA tensor; it is copied to the device as
    float32 and handed to rr_setup_dense."""

    def __init__(self, X, n_clusters=0, seed=0, kmeans_max_iter=0, labels=None, lambda_slots=0,
                 autotune=False, device="cuda"):
        import numpy as np
        import torch
        self.device = torch.device(device)
        Xt = torch.as_tensor(X, dtype=torch.float32, device=self.device).contiguous()
        self.N, self.F = Xt.shape
        lab = None
        nlab = 0
        if labels is not None:
            lab = torch.as_tensor(np.asarray(labels, dtype=np.int32), device=self.device)
            nlab = int(np.max(labels)) + 1 if len(labels) else 1
        self.h = rr_setup_dense(Xt, n_clusters, seed, kmeans_max_iter, lab, nlab, lambda_slots, autotune)
        torch.cuda.current_stream().synchronize()
        del Xt
        self.info = rr_get_setup_info(self.h)

    def _block(self, v, n):
        import torch
        t = torch.as_tensor(v, dtype=torch.float64, device=self.device)
        if t.dim() == 1:
            t = t[None, :]
        t = t.contiguous()
        if t.shape[1] != n:
            raise ValueError(f"expected rows of {n} entries")
        return t

    def solve_block(self, lam, Y, rhs_is_b=False, **kw):
        """Y: (m, N) targets (or (m, F) right-hand sides); returns (W (m, F), infos)."""
        import torch
        rhs = self._block(Y, self.F if rhs_is_b else self.N)
        w = torch.empty(rhs.shape[0], self.F, dtype=torch.float64, device=self.device)
        st, infos = rr_solve_block(self.h, lam, rhs, w, rhs_is_b=rhs_is_b, **kw)
        return w, infos

    def solve(self, lam, y, rhs_is_b=False, **kw):
        w, infos = self.solve_block(lam, y, rhs_is_b=rhs_is_b, **kw)
        return w[0], infos[0]

    def apply_operator_block(self, lam, V, precision="f64"):
        import torch
        v = self._block(V, self.F)
        q = torch.empty_like(v)
        rr_apply_operator_block(self.h, lam, v, q, precision)
        return q

    def apply_operator(self, lam, v):
        return self.apply_operator_block(lam, v)[0]
