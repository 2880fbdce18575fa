"""Python binding of the libhmx C ABI (``include/hmx.h``).

Argument marshalling only: every step of the build and the matvec runs in the
HIP kernels of ``libhmx.so``.  PyTorch supplies device memory (tensors) and
streams.  The functions carry the C names; ``HMatrix`` is a small owner of a
handle.  There is no CPU fallback: if the library is missing this module
raises on import of the library.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhmx.so")

HMX_OK, HMX_ERR_INVALID_ARG, HMX_ERR_OOM, HMX_ERR_DEVICE, HMX_ERR_NOT_CONVERGED, \
    HMX_ERR_UNSUPPORTED = range(6)
HMX_F64, HMX_F32, HMX_BF16 = 0, 1, 2
HMX_GAUSSIAN, HMX_MATERN32, HMX_MATERN_NU1, HMX_TEST_CONST, HMX_TEST_LOWRANK = 0, 1, 2, 3, 4
HMX_RANK_ADAPTIVE, HMX_RANK_LEARNED, HMX_RANK_FIXED = 0, 1, 2
HMX_MLP_NPARAMS, HMX_MLP_FEATURES = 8961, 8
RANK_MODES = {"adaptive": HMX_RANK_ADAPTIVE, "learned": HMX_RANK_LEARNED, "fixed": HMX_RANK_FIXED}
KERNELS = {"gaussian": HMX_GAUSSIAN, "matern32": HMX_MATERN32, "matern_nu1": HMX_MATERN_NU1,
           "const": HMX_TEST_CONST,
           "lowrank": HMX_TEST_LOWRANK}
DTYPES = {"f64": HMX_F64, "f32": HMX_F32, "bf16": HMX_BF16}

# every symbol declared in include/hmx.h
EXPORTS = ["hmx_params_default", "hmx_build", "hmx_matvec", "hmx_cg_solve", "hmx_get_partition",
           "hmx_get_boxes", "hmx_get_ranks", "hmx_get_factors", "hmx_get_stats",
           "hmx_profile_begin", "hmx_profile_end", "hmx_destroy", "hmx_trim",
           "hmx_status_string", "hmx_last_error", "hmx_mlp_create", "hmx_mlp_destroy",
           "hmx_mlp_set_params", "hmx_mlp_get_params", "hmx_mlp_fit_normalization",
           "hmx_mlp_forward", "hmx_mlp_loss_grad", "hmx_mlp_adam", "hmx_mlp_train",
           "hmx_block_features", "hmx_build_batched", "hmx_get_batch", "hmx_matvec_graph",
           "hmx_graph_launch", "hmx_graph_destroy", "hmx_autotune", "hmx_set_tile_config",
           "hmx_rank_predict", "hmx_cg_solve_noalloc", "hmx_matvec_batched", "hmx_mlp_save",
           "hmx_mlp_load", "hmx_build_rect", "hmx_matmat"]
HMX_CG_NOALLOC_MAX_BYTES = 50397184
HMX_TILE_CONFIGS = 18


class hmx_kernel(C.Structure):
    _fields_ = [("kind", C.c_int), ("p0", C.c_double), ("p1", C.c_double)]


# device allocator hooks of hmx_params (dev_alloc / dev_free)
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p)


class hmx_params(C.Structure):
    _fields_ = [("leaf_size", C.c_int32), ("eta", C.c_double), ("aca_eps", C.c_double),
                ("aca_eta", C.c_double), ("aca_eps0", C.c_double), ("max_rank", C.c_int32),
                ("sigma2", C.c_double), ("compute_dtype", C.c_int), ("storage_dtype", C.c_int),
                ("near_dtype", C.c_int),
                ("rank_mode", C.c_int), ("aca_chunk_mb", C.c_int32),
                ("aca_only", C.c_int32), ("mlp", C.c_void_p),
                ("learned_one_shot", C.c_int32), ("near_recompute", C.c_int32),
                ("aca_split_rows", C.c_int32), ("symmetric_far", C.c_int32),
                ("dev_alloc", ALLOC_FN), ("dev_free", FREE_FN), ("alloc_ctx", C.c_void_p),
                ("far_recompute", C.c_int32)]


class hmx_stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("d", C.c_int32), ("levels", C.c_int32),
                ("n_adm", C.c_int64), ("n_dense", C.c_int64), ("n_tiles", C.c_int64),
                ("sum_rank", C.c_int64), ("max_rank_used", C.c_int32),
                ("entry_bytes", C.c_int32), ("factor_entries", C.c_int64),
                ("u_entries", C.c_int64), ("v_entries", C.c_int64),
                ("near_entries", C.c_int64), ("aca_columns", C.c_int64),
                ("aca_chunks", C.c_int64), ("near_entry_bytes", C.c_int32),
                ("tile_config", C.c_int32), ("matvec_bytes", C.c_double),
                ("phase_ms", C.c_double * 8),
                ("device_bytes", C.c_int64), ("level_sizes", C.c_int64 * 64),
                ("aca_fallback", C.c_int64), ("aca_capacity", C.c_int64),
                ("predict_ms", C.c_double), ("aca_overflow", C.c_int64),
                ("aca_kernel_evals", C.c_int64), ("aca_flops", C.c_double),
                ("rows", C.c_int64), ("cols", C.c_int64),
                ("alloc_fresh_bytes", C.c_int64), ("alloc_flushes", C.c_int64)]


class HmxError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("hmx status %d (%s): %s" % (status, _status_name(status), msg))
        self.status = status


def _status_name(s):
    return ["ok", "invalid argument", "out of device memory", "device error",
            "not converged", "unsupported"][s] if 0 <= s < 6 else "unknown"


_lib = None


def lib():
    """Load libhmx.so (import torch first so both share one HIP runtime)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libhmx.so is not built (%s); run __graft_entry__.build()"
                               % LIB_PATH)
        try:
            import torch  # noqa: F401  (loads the HIP runtime the library binds to)
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        P, i32, i64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.hmx_params_default.argtypes = [C.POINTER(hmx_params)]
        L.hmx_build.argtypes = [P, C.c_int, i64, i32, C.POINTER(hmx_kernel),
                                C.POINTER(hmx_params), P, C.POINTER(P)]
        L.hmx_matvec.argtypes = [P, P, P, C.c_int, f64, f64, P]
        L.hmx_cg_solve.argtypes = [P, P, P, f64, i32, P, C.POINTER(i32), C.POINTER(f64),
                                   C.POINTER(f64)]
        L.hmx_cg_solve_noalloc.argtypes = [P, P, P, f64, i32, P, C.POINTER(i32), C.POINTER(f64),
                                           C.POINTER(f64)]
        L.hmx_matvec_batched.argtypes = [i32, P, P, P, C.c_int, f64, f64, P]
        L.hmx_matmat.argtypes = [P, P, i64, P, i64, i32, C.c_int, f64, f64, P]
        L.hmx_build_rect.argtypes = [P, i64, P, i64, C.c_int, i32, C.POINTER(hmx_kernel),
                                     C.POINTER(hmx_params), P, C.POINTER(P)]
        L.hmx_mlp_save.argtypes = [P, C.c_char_p]
        L.hmx_mlp_load.argtypes = [C.c_char_p, C.POINTER(P)]
        L.hmx_get_partition.argtypes = [P, P, P, P, C.POINTER(i64), P, C.POINTER(i64), P]
        L.hmx_get_boxes.argtypes = [P, P, P, P]
        L.hmx_get_ranks.argtypes = [P, P, P]
        L.hmx_get_factors.argtypes = [P, i64, P, P, C.POINTER(i32), P]
        L.hmx_get_stats.argtypes = [P, C.POINTER(hmx_stats)]
        L.hmx_destroy.argtypes = [P]
        L.hmx_trim.argtypes = [C.POINTER(i64)]
        L.hmx_profile_begin.argtypes = [P, i32]
        L.hmx_profile_end.argtypes = [P, P, C.POINTER(i32)]
        L.hmx_mlp_create.argtypes = [P, C.POINTER(P)]
        L.hmx_mlp_destroy.argtypes = [P]
        L.hmx_mlp_set_params.argtypes = [P, P, P, P]
        L.hmx_mlp_get_params.argtypes = [P, P, P, P]
        L.hmx_mlp_fit_normalization.argtypes = [P, P, i64, P]
        L.hmx_mlp_forward.argtypes = [P, P, i64, P, P]
        L.hmx_mlp_loss_grad.argtypes = [P, P, P, i64, f64, P, C.POINTER(f64), P]
        L.hmx_mlp_adam.argtypes = [P, P, f64, f64, f64, f64, P]
        L.hmx_mlp_train.argtypes = [P, P, P, i64, P, i64, i32, f64, f64, P, P]
        L.hmx_block_features.argtypes = [P, P, P, C.POINTER(i64), P]
        L.hmx_rank_predict.argtypes = [P, P, P, P, C.POINTER(i64), P]
        L.hmx_build_batched.argtypes = [i32, P, C.c_int, P, P, P, C.POINTER(hmx_params), P,
                                        C.POINTER(P)]
        L.hmx_get_batch.argtypes = [P, C.POINTER(i32), P]
        L.hmx_matvec_graph.argtypes = [P, P, P, C.c_int, f64, f64, i32, C.POINTER(P)]
        L.hmx_graph_launch.argtypes = [P, P]
        L.hmx_graph_destroy.argtypes = [P]
        L.hmx_autotune.argtypes = [P, i32, P, C.POINTER(i32), P]
        L.hmx_set_tile_config.argtypes = [P, i32]
        L.hmx_status_string.restype = C.c_char_p
        L.hmx_status_string.argtypes = [C.c_int]
        L.hmx_last_error.restype = C.c_char_p
        L.hmx_last_error.argtypes = []
        for name in EXPORTS:
            getattr(L, name).restype = getattr(L, name).restype if name in (
                "hmx_status_string", "hmx_last_error") else C.c_int
        _lib = L
    return _lib


def _check(status):
    if status != HMX_OK:
        raise HmxError(status, lib().hmx_last_error().decode())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _dtype_of(t):
    import torch
    if t.dtype == torch.float64:
        return HMX_F64
    if t.dtype == torch.float32:
        return HMX_F32
    if t.dtype == torch.bfloat16:
        return HMX_BF16
    raise TypeError("unsupported dtype %s" % t.dtype)


def hmx_params_default(**overrides) -> hmx_params:
    p = hmx_params()
    _check(lib().hmx_params_default(C.byref(p)))
    for k, v in overrides.items():
        if k in ("compute_dtype", "storage_dtype", "near_dtype") and isinstance(v, str):
            v = DTYPES[v]
        if k == "rank_mode" and isinstance(v, str):
            v = RANK_MODES[v]
        if k == "mlp":
            v = v.handle if isinstance(v, RankMLP) else v
        if k == "allocator":  # a TorchAllocator (or any object with alloc_fn / free_fn)
            p.dev_alloc, p.dev_free = v.alloc_fn, v.free_fn
            continue
        setattr(p, k, v)
    if "compute_dtype" in overrides and "storage_dtype" not in overrides:
        p.storage_dtype = p.compute_dtype  # store in the compute precision unless asked
    if "near_dtype" not in overrides:
        p.near_dtype = p.storage_dtype
    return p


def make_kernel(kind, p0=1.0) -> hmx_kernel:
    return hmx_kernel(KERNELS[kind] if isinstance(kind, str) else int(kind), float(p0), 0.0)


def hmx_build(points, kernel: hmx_kernel, params: hmx_params, stream=None):
    """points: contiguous CUDA tensor (n, d) float64/float32.  Returns a handle."""
    if not points.is_cuda or not points.is_contiguous() or points.dim() != 2:
        raise ValueError("points must be a contiguous (n, d) device tensor")
    h = C.c_void_p()
    _check(lib().hmx_build(C.c_void_p(points.data_ptr()), _dtype_of(points), points.shape[0],
                           points.shape[1], C.byref(kernel), C.byref(params), _stream(stream),
                           C.byref(h)))
    return h


def _check_vectors(h, *vecs, lengths=None):
    """The C ABI takes bare device pointers: every vector must be a
    contiguous device tensor of exactly the length the handle expects (its n,
    or per vector `lengths`), all of one dtype and on one device (a short
    vector would be read and written past its end by the gather and scatter
    kernels)."""
    n = hmx_get_stats(h).n
    lengths = lengths or [n] * len(vecs)
    t0 = vecs[0]
    for t, m in zip(vecs, lengths):
        if not (t.is_cuda and t.is_contiguous()):
            raise ValueError("vectors must be contiguous device tensors")
        if t.dim() != 1 or t.numel() != m:
            raise ValueError("vectors must have shape (%d,), got %s" % (m, tuple(t.shape)))
        if t.dtype != t0.dtype or t.device != t0.device:
            raise ValueError("vectors must share one dtype and device")


def _shape(h):
    """(rows, cols) of the handle's matrix."""
    st = hmx_get_stats(h)
    return int(st.rows), int(st.cols)


def hmx_matvec(h, x, z, alpha=1.0, beta=0.0, stream=None):
    rows, cols = _shape(h)
    _check_vectors(h, x, z, lengths=(cols, rows))
    _check(lib().hmx_matvec(h, C.c_void_p(x.data_ptr()), C.c_void_p(z.data_ptr()), _dtype_of(x),
                            float(alpha), float(beta), _stream(stream)))


def hmx_matmat(h, X, Z, alpha=1.0, beta=0.0, stream=None):
    """Z = alpha (H + sigma2 I) X + beta Z for several right-hand sides.  X:
    contiguous (m, ldx) device tensor with ldx >= cols (right-hand side c in
    X[c, :cols]), Z: (m, ldz) with ldz >= rows; the C ABI sees them as
    column-major cols x m and rows x m with leading dimensions ldx, ldz."""
    rows, cols = _shape(h)
    for t, w in ((X, cols), (Z, rows)):
        if not (t.is_cuda and t.is_contiguous()) or t.dim() != 2 or t.shape[1] < w:
            raise ValueError("X must be a contiguous (m, >= %d) and Z a (m, >= %d) device tensor"
                             % (cols, rows))
    if X.shape[0] != Z.shape[0] or X.dtype != Z.dtype or X.device != Z.device:
        raise ValueError("X and Z need the same number of rows, dtype and device")
    _check(lib().hmx_matmat(h, C.c_void_p(X.data_ptr()), int(X.shape[1]),
                            C.c_void_p(Z.data_ptr()), int(Z.shape[1]), int(X.shape[0]),
                            _dtype_of(X), float(alpha), float(beta), _stream(stream)))


def hmx_matvec_batched(handles, xs, zs, alpha=1.0, beta=0.0, stream=None):
    """z[q] = alpha (H_q + sigma2 I) x[q] + beta z[q] over separately built handles."""
    if not (len(handles) == len(xs) == len(zs)):
        raise ValueError("handles, xs and zs must have one entry per problem")
    for h, x, z in zip(handles, xs, zs):
        rows, cols = _shape(h)
        _check_vectors(h, x, z, lengths=(cols, rows))
    k = len(handles)
    hs = (C.c_void_p * k)(*[h.value if isinstance(h, C.c_void_p) else h for h in handles])
    xp = (C.c_void_p * k)(*[x.data_ptr() for x in xs])
    zp = (C.c_void_p * k)(*[z.data_ptr() for z in zs])
    _check(lib().hmx_matvec_batched(k, hs, xp, zp, _dtype_of(xs[0]) if k else HMX_F32,
                                    float(alpha), float(beta), _stream(stream)))


def hmx_cg_solve(h, b, x, rel_tol=1e-6, max_iter=1000, stream=None, raise_on_fail=True,
                 noalloc=False):
    """Solve (H + sigma2 I) x = b by CG.  Returns (status, iters, rel_res, true_rel_res).
    noalloc=True calls hmx_cg_solve_noalloc (fixed work space, no allocation)."""
    _check_vectors(h, b, x)
    it, rr, tr = C.c_int32(0), C.c_double(0), C.c_double(0)
    fn = lib().hmx_cg_solve_noalloc if noalloc else lib().hmx_cg_solve
    s = fn(h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), float(rel_tol), int(max_iter),
           _stream(stream), C.byref(it), C.byref(rr), C.byref(tr))
    if s not in (HMX_OK, HMX_ERR_NOT_CONVERGED) or (raise_on_fail and s != HMX_OK):
        _check(s)
    return s, it.value, rr.value, tr.value


def hmx_get_stats(h) -> hmx_stats:
    s = hmx_stats()
    _check(lib().hmx_get_stats(h, C.byref(s)))
    return s


def hmx_get_partition(h, stream=None):
    s = hmx_get_stats(h)
    n = s.n
    codes = np.empty(n, np.uint64)
    perm = np.empty(n, np.int32)
    na, nd = C.c_int64(s.n_adm), C.c_int64(s.n_dense)
    adm = np.empty((max(s.n_adm, 1), 5), np.int32)
    den = np.empty((max(s.n_dense, 1), 5), np.int32)
    _check(lib().hmx_get_partition(h, codes.ctypes.data_as(C.c_void_p),
                                   perm.ctypes.data_as(C.c_void_p), adm.ctypes.data_as(C.c_void_p),
                                   C.byref(na), den.ctypes.data_as(C.c_void_p), C.byref(nd),
                                   _stream(stream)))
    return dict(codes=codes, perm=perm, adm=adm[: na.value].copy(), dense=den[: nd.value].copy(),
                level_sizes=np.array(s.level_sizes[: s.levels], np.int64))


def hmx_get_boxes(h, stream=None):
    s = hmx_get_stats(h)
    d = s.d
    gb = np.empty(2 * d)
    lb = np.empty((s.n_tiles, 2 * d + 2))
    _check(lib().hmx_get_boxes(h, gb.ctypes.data_as(C.c_void_p), lb.ctypes.data_as(C.c_void_p),
                               _stream(stream)))
    return gb[:d].copy(), gb[d:].copy(), lb


def hmx_get_ranks(h, stream=None):
    s = hmx_get_stats(h)
    r = np.zeros(max(s.n_adm, 1), np.int32)
    _check(lib().hmx_get_ranks(h, r.ctypes.data_as(C.c_void_p), _stream(stream)))
    return r[: s.n_adm].copy()


def hmx_get_factors(h, leaf: int, m: int, n: int, kmax: int, stream=None):
    U = np.zeros(m * kmax)
    V = np.zeros(n * kmax)
    r = C.c_int32(0)
    _check(lib().hmx_get_factors(h, int(leaf), U.ctypes.data_as(C.c_void_p),
                                 V.ctypes.data_as(C.c_void_p), C.byref(r), _stream(stream)))
    k = r.value
    return U[: k * m].reshape(k, m).T.copy(), V[: k * n].reshape(k, n).T.copy(), k


def hmx_profile_begin(h, max_calls: int):
    _check(lib().hmx_profile_begin(h, int(max_calls)))


def hmx_profile_end(h):
    """Returns (summed ms per phase [gather, phase1, rowtile], calls)."""
    ms = np.zeros(3)
    calls = C.c_int32(0)
    _check(lib().hmx_profile_end(h, ms.ctypes.data_as(C.c_void_p), C.byref(calls)))
    return ms, calls.value


def hmx_destroy(h):
    if h:
        _check(lib().hmx_destroy(h))


def hmx_trim() -> int:
    """Return the library's cached device blocks to the driver; bytes freed."""
    r = C.c_int64(0)
    _check(lib().hmx_trim(C.byref(r)))
    return r.value


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _np_f32(a, n):
    a = np.ascontiguousarray(a, dtype=np.float32).reshape(-1)
    if a.shape[0] != n:
        raise ValueError("expected %d values, got %d" % (n, a.shape[0]))
    return a


def hmx_mlp_create(params=None):
    h = C.c_void_p()
    w = None if params is None else _np_f32(params, HMX_MLP_NPARAMS)
    _check(lib().hmx_mlp_create(None if w is None else w.ctypes.data_as(C.c_void_p), C.byref(h)))
    return h


def hmx_mlp_destroy(h):
    if h:
        _check(lib().hmx_mlp_destroy(h))


def hmx_mlp_save(h, path):
    _check(lib().hmx_mlp_save(h, os.fsencode(path)))


def hmx_mlp_load(path):
    h = C.c_void_p()
    _check(lib().hmx_mlp_load(os.fsencode(path), C.byref(h)))
    return h


def hmx_mlp_set_params(h, params=None, mean=None, scale=None):
    w = None if params is None else _np_f32(params, HMX_MLP_NPARAMS)
    mu = None if mean is None else _np_f32(mean, HMX_MLP_FEATURES)
    sc = None if scale is None else _np_f32(scale, HMX_MLP_FEATURES)
    _check(lib().hmx_mlp_set_params(h, *[None if a is None else a.ctypes.data_as(C.c_void_p)
                                         for a in (w, mu, sc)]))


def hmx_mlp_get_params(h):
    w = np.empty(HMX_MLP_NPARAMS, np.float32)
    mu = np.empty(HMX_MLP_FEATURES, np.float32)
    sc = np.empty(HMX_MLP_FEATURES, np.float32)
    _check(lib().hmx_mlp_get_params(h, *[a.ctypes.data_as(C.c_void_p) for a in (w, mu, sc)]))
    return w, mu, sc


def _dev_f32(t, cols=None):
    import torch
    if not (t.is_cuda and t.is_contiguous() and t.dtype == torch.float32):
        raise ValueError("expected a contiguous float32 device tensor")
    if cols is not None and (t.dim() != 2 or t.shape[1] != cols):
        raise ValueError("expected shape (B, %d)" % cols)
    return t


def hmx_mlp_fit_normalization(h, X, stream=None):
    _dev_f32(X, HMX_MLP_FEATURES)
    _check(lib().hmx_mlp_fit_normalization(h, _ptr(X), X.shape[0], _stream(stream)))


def hmx_mlp_forward(h, X, out=None, stream=None):
    import torch
    _dev_f32(X, HMX_MLP_FEATURES)
    if out is None:
        out = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    _check(lib().hmx_mlp_forward(h, _ptr(X), X.shape[0], _ptr(out), _stream(stream)))
    return out


def hmx_mlp_loss_grad(h, X, y, q=0.9, grad=None, stream=None):
    """Returns (loss, grad tensor)."""
    import torch
    _dev_f32(X, HMX_MLP_FEATURES)
    _dev_f32(y)
    if grad is None:
        grad = torch.empty(HMX_MLP_NPARAMS, dtype=torch.float32, device=X.device)
    loss = C.c_double(0)
    _check(lib().hmx_mlp_loss_grad(h, _ptr(X), _ptr(y), X.shape[0], float(q), _ptr(grad),
                                   C.byref(loss), _stream(stream)))
    return loss.value, grad


def hmx_mlp_adam(h, grad, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _dev_f32(grad)
    _check(lib().hmx_mlp_adam(h, _ptr(grad), float(lr), float(beta1), float(beta2), float(eps),
                              _stream(stream)))


def hmx_mlp_train(h, X, y, batch_idx, batch, steps, q=0.9, lr=1e-3, losses=None, stream=None):
    import torch
    _dev_f32(X, HMX_MLP_FEATURES)
    _dev_f32(y)
    if not (batch_idx.is_cuda and batch_idx.dtype == torch.int64 and batch_idx.is_contiguous()):
        raise ValueError("batch_idx must be a contiguous int64 device tensor")
    if batch_idx.numel() < int(batch) * int(steps):
        raise ValueError("batch_idx holds fewer than batch * steps indices")
    if losses is not None and (losses.dtype != torch.float64 or losses.numel() < steps):
        raise ValueError("losses must be a float64 device tensor of >= steps entries")
    _check(lib().hmx_mlp_train(h, _ptr(X), _ptr(y), X.shape[0], _ptr(batch_idx), int(batch),
                               int(steps), float(q), float(lr), _ptr(losses), _stream(stream)))


def hmx_block_features(h, with_ranks=True, stream=None):
    """(features (n_adm, 8) float32, ranks (n_adm,) float32 or None) as device tensors."""
    import torch
    s = hmx_get_stats(h)
    na = C.c_int64(s.n_adm)
    F = torch.empty((max(s.n_adm, 1), HMX_MLP_FEATURES), dtype=torch.float32, device="cuda")
    y = torch.empty(max(s.n_adm, 1), dtype=torch.float32, device="cuda") if with_ranks else None
    _check(lib().hmx_block_features(h, _ptr(F), _ptr(y), C.byref(na), _stream(stream)))
    return F[: na.value], (y[: na.value] if y is not None else None)


def hmx_rank_predict(h, mlp, stream=None):
    """The fused in-build inference on the handle's admissible leaves:
    (raw predictions (n_adm,) float32, targets (n_adm,) int32) device tensors."""
    import torch
    s = hmx_get_stats(h)
    na = C.c_int64(s.n_adm)
    pred = torch.empty(max(s.n_adm, 1), dtype=torch.float32, device="cuda")
    tgt = torch.empty(max(s.n_adm, 1), dtype=torch.int32, device="cuda")
    m = mlp.handle if isinstance(mlp, RankMLP) else mlp
    _check(lib().hmx_rank_predict(h, m, _ptr(pred), _ptr(tgt), C.byref(na), _stream(stream)))
    return pred[: na.value], tgt[: na.value]


def hmx_matvec_graph(h, x, z, alpha=1.0, beta=0.0, reps=1):
    """Capture reps matvecs into a HIP graph; returns the graph handle."""
    rows, cols = _shape(h)
    _check_vectors(h, x, z, lengths=(cols, rows))
    g = C.c_void_p()
    _check(lib().hmx_matvec_graph(h, C.c_void_p(x.data_ptr()), C.c_void_p(z.data_ptr()),
                                  _dtype_of(x), float(alpha), float(beta), int(reps),
                                  C.byref(g)))
    return g


def hmx_graph_launch(g, stream=None):
    _check(lib().hmx_graph_launch(g, _stream(stream)))


def hmx_graph_destroy(g):
    if g:
        _check(lib().hmx_graph_destroy(g))


def hmx_autotune(h, reps=5, stream=None):
    """Returns (chosen configuration, mean ms per configuration)."""
    ch = C.c_int32(-1)
    t = np.zeros(HMX_TILE_CONFIGS)
    _check(lib().hmx_autotune(h, int(reps), _stream(stream), C.byref(ch),
                              t.ctypes.data_as(C.c_void_p)))
    return ch.value, t


def hmx_set_tile_config(h, config):
    _check(lib().hmx_set_tile_config(h, int(config)))


def hmx_build_batched(points_list, kernels, params: hmx_params, stream=None):
    """points_list: device tensors (n_p, d_p), all float32 or all float64;
    kernels: hmx_kernel per problem.  Returns (handle, offsets)."""
    np_ = len(points_list)
    if np_ < 1 or len(kernels) != np_:
        raise ValueError("need one kernel per problem")
    dt = _dtype_of(points_list[0])
    for t in points_list:
        if not t.is_cuda or not t.is_contiguous() or t.dim() != 2 or _dtype_of(t) != dt:
            raise ValueError("points must be contiguous (n, d) device tensors of one dtype")
    ptrs = (C.c_void_p * np_)(*[t.data_ptr() for t in points_list])
    ns = (C.c_int64 * np_)(*[t.shape[0] for t in points_list])
    ds = (C.c_int32 * np_)(*[t.shape[1] for t in points_list])
    ks = (hmx_kernel * np_)(*kernels)
    h = C.c_void_p()
    _check(lib().hmx_build_batched(np_, ptrs, dt, ns, ds, ks, C.byref(params), _stream(stream),
                                   C.byref(h)))
    return h, hmx_get_batch(h)


def hmx_build_rect(rows_pts, cols_pts, kernel: hmx_kernel, params: hmx_params, stream=None):
    """Rectangular H-matrix of A(Y1 x Y2): rows_pts (n1, d) and cols_pts (n2, d)
    contiguous device tensors of one float dtype."""
    dt = _dtype_of(rows_pts)
    for t in (rows_pts, cols_pts):
        if not t.is_cuda or not t.is_contiguous() or t.dim() != 2 or _dtype_of(t) != dt:
            raise ValueError("points must be contiguous (n, d) device tensors of one dtype")
    if rows_pts.shape[1] != cols_pts.shape[1]:
        raise ValueError("both point sets need the same dimension")
    h = C.c_void_p()
    _check(lib().hmx_build_rect(_ptr(rows_pts), int(rows_pts.shape[0]), _ptr(cols_pts),
                                int(cols_pts.shape[0]), dt, int(rows_pts.shape[1]),
                                C.byref(kernel), C.byref(params), _stream(stream), C.byref(h)))
    return h


def hmx_get_batch(h):
    """Problem offsets (nprob + 1 entries)."""
    nprob = C.c_int32(0)
    _check(lib().hmx_get_batch(h, C.byref(nprob), None))
    off = np.zeros(nprob.value + 1, np.int64)
    _check(lib().hmx_get_batch(h, C.byref(nprob), off.ctypes.data_as(C.c_void_p)))
    return off


class TorchAllocator:
    """Device allocator hooks that take the library's device memory from
    PyTorch's caching allocator (pass as ``allocator=`` to a build).  Keeps
    the ctypes callbacks alive and counts what is outstanding."""

    def __init__(self, device=None):
        import torch
        self._torch = torch
        self.device = torch.cuda.current_device() if device is None else device
        self.live = {}          # pointer -> bytes
        self.allocs = 0
        self.frees = 0
        self.alloc_fn = ALLOC_FN(self._alloc)
        self.free_fn = FREE_FN(self._free)

    def take(self, nbytes):
        """Allocate nbytes of device memory; return the pointer or None."""
        try:
            return self._torch.cuda.caching_allocator_alloc(nbytes, self.device)
        except RuntimeError:  # torch's out-of-memory error
            return None

    def _alloc(self, nbytes, ctx):
        self.allocs += 1
        ptr = self.take(int(nbytes))
        if ptr:
            self.live[ptr] = int(nbytes)
        return ptr

    def _free(self, ptr, nbytes, ctx):
        self.frees += 1
        size = self.live.pop(ptr, None)
        if size != int(nbytes):
            raise RuntimeError("dev_free of %s (%d bytes) that was not handed out" % (ptr, nbytes))
        self._torch.cuda.caching_allocator_delete(ptr)

    @property
    def outstanding_bytes(self):
        return sum(self.live.values())


class RankMLP:
    """Owner of an hmx_mlp rank predictor."""

    def __init__(self, params=None):
        self.handle = hmx_mlp_create(params)

    @classmethod
    def load(cls, path):
        """A predictor from a checkpoint file written by save()."""
        self = cls.__new__(cls)
        self.handle = hmx_mlp_load(path)
        return self

    def save(self, path):
        hmx_mlp_save(self.handle, path)

    def set_params(self, params=None, mean=None, scale=None):
        hmx_mlp_set_params(self.handle, params, mean, scale)

    def get_params(self):
        return hmx_mlp_get_params(self.handle)

    def fit_normalization(self, X, stream=None):
        hmx_mlp_fit_normalization(self.handle, X, stream)

    def forward(self, X, stream=None):
        return hmx_mlp_forward(self.handle, X, stream=stream)

    def loss_grad(self, X, y, q=0.9, stream=None):
        return hmx_mlp_loss_grad(self.handle, X, y, q, stream=stream)

    def adam(self, grad, lr=1e-3, stream=None):
        hmx_mlp_adam(self.handle, grad, lr, stream=stream)

    def train(self, X, y, batch_idx, batch, steps, q=0.9, lr=1e-3, losses=None, stream=None):
        hmx_mlp_train(self.handle, X, y, batch_idx, batch, steps, q, lr, losses, stream)

    def close(self):
        if self.handle:
            hmx_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HMatrix:
    """Owner of an hmx handle built from device points."""

    def __init__(self, points, kernel="gaussian", p0=1.0, stream=None, **params):
        self.params = hmx_params_default(**params)
        self.allocator = params.get("allocator")  # its callbacks must outlive the handle
        self.kernel = make_kernel(kernel, p0)
        self.n, self.d = int(points.shape[0]), int(points.shape[1])
        self.h = hmx_build(points, self.kernel, self.params, stream)
        self.offsets = np.array([0, self.n], np.int64)

    @classmethod
    def batched(cls, points_list, kernel="gaussian", p0s=None, stream=None, **params):
        """One block-diagonal handle over many problems (hmx_build_batched)."""
        self = cls.__new__(cls)
        self.params = hmx_params_default(**params)
        self.allocator = params.get("allocator")
        p0s = [1.0] * len(points_list) if p0s is None else p0s
        ks = [make_kernel(kernel, p) for p in p0s]
        self.kernel = ks[0]
        self.h, self.offsets = hmx_build_batched(points_list, ks, self.params, stream)
        self.n, self.d = int(self.offsets[-1]), 3
        return self

    @classmethod
    def rect(cls, rows_pts, cols_pts, kernel="gaussian", p0=1.0, stream=None, **params):
        """The rectangular matrix A(Y1 x Y2) (hmx_build_rect)."""
        self = cls.__new__(cls)
        self.params = hmx_params_default(**params)
        self.allocator = params.get("allocator")
        self.kernel = make_kernel(kernel, p0)
        self.h = hmx_build_rect(rows_pts, cols_pts, self.kernel, self.params, stream)
        self.offsets = hmx_get_batch(self.h)
        self.n, self.d = int(self.offsets[-1]), int(rows_pts.shape[1])
        return self

    def matvec(self, x, z=None, alpha=1.0, beta=0.0, stream=None):
        import torch
        if z is None:
            rows, _ = _shape(self.h)
            z = torch.empty(rows, dtype=x.dtype, device=x.device)
        hmx_matvec(self.h, x, z, alpha, beta, stream)
        return z

    def matmat(self, X, Z=None, alpha=1.0, beta=0.0, stream=None):
        """Several right-hand sides, one per row of X."""
        import torch
        if Z is None:
            rows, _ = _shape(self.h)
            Z = torch.empty((X.shape[0], rows), dtype=X.dtype, device=X.device)
        hmx_matmat(self.h, X, Z, alpha, beta, stream)
        return Z

    def stats(self):
        return hmx_get_stats(self.h)

    def partition(self):
        return hmx_get_partition(self.h)

    def ranks(self):
        return hmx_get_ranks(self.h)

    def close(self):
        if self.h:
            hmx_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
