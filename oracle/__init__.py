"""CPU oracle for the H-matrix path (TEST INFRASTRUCTURE ONLY).

Plain FP64 C code (``hmxo.c``) written from the paper's definitions, wrapped
with ctypes.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import this package.  It shares no code with the HIP
library in ``paper_1708_09707_amd``; the only common module is ``synth``, which
draws random inputs and holds none of the method's arithmetic.

Parity pins for every function live in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hmxo.c")
_LIB = os.path.join(_HERE, "libhmxo.so")

GAUSSIAN, MATERN32, MATERN_NU1, CONST, LOWRANK = 0, 1, 2, 3, 4
KINDS = {"gaussian": GAUSSIAN, "matern32": MATERN32, "matern_nu1": MATERN_NU1, "const": CONST,
         "lowrank": LOWRANK}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd, cwd=_HERE)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.c_void_p
        i32, i64, f64 = C.c_int32, C.c_int64, C.c_double
        L.hmxo_kernel.restype = f64
        L.hmxo_kernel.argtypes = [C.c_int, f64, P, P, C.c_int]
        L.hmxo_dense_matmat.argtypes = [P, i64, i32, i32, f64, f64, P, i32, P, i64, P]
        L.hmxo_xk1.restype = f64
        L.hmxo_xk1.argtypes = [f64]
        L.hmxo_global_box.argtypes = [P, i64, i32, P, P]
        L.hmxo_morton.argtypes = [P, i64, i32, P, P, P]
        L.hmxo_sort.argtypes = [P, i64, P]
        L.hmxo_ordered_coords.argtypes = [P, i64, i32, P, P]
        L.hmxo_cluster_tree.restype = i64
        L.hmxo_cluster_tree.argtypes = [i64, i32, i64, P, P, P, P]
        L.hmxo_boxes.argtypes = [P, i64, i32, i64, P, P, P, P]
        L.hmxo_admissible.argtypes = [P, P, P, P, i32, f64]
        L.hmxo_partition.argtypes = [P, i64, i32, i32, f64, i64, P, P, i64, P, P, P, P]
        L.hmxo_aca.argtypes = [P, i64, i32, i32, f64, i64, i64, i64, i64, i32, f64, f64, f64,
                               i32, i32, P, P, P, P]
        L.hmxo_aca_traced.argtypes = L.hmxo_aca.argtypes + [P]
        L.hmxo_hmvp.argtypes = [P, i64, i32, i32, f64, i32, f64, i32, f64, f64, f64, i32, f64,
                                f64, f64, P, P, i64, P, P]
        L.hmxo_hmvp_ex.argtypes = [P, i64, i32, i32, f64, i32, f64, i32, f64, f64, f64, i32, i32,
                                   f64, f64, f64, P, P, i64, P, P]
        L.hmxo_dense_matvec.argtypes = [P, i64, i32, i32, f64, f64, P, P, i64, P]
        L.hmxo_dense_matvec_rect.argtypes = [P, i64, P, i64, i32, i32, f64, P, P]
        L.hmxo_partition_rect.argtypes = [P, i64, P, i64, i32, i32, f64, i64, P, P, i64, P, P,
                                          P, P]
        L.hmxo_hmvp_rect.argtypes = [P, i64, P, i64, i32, i32, f64, i32, f64, i32, f64, f64, f64,
                                     i32, f64, f64, P, P, i64, P, P]
        L.hmxo_dense_block.argtypes = [P, i64, i32, i32, f64, i64, i64, i64, i64, P]
        L.hmxo_hmvp_rows.argtypes = [P, i64, i32, i32, f64, i32, f64, i32, f64, f64, f64, i32,
                                     i64, i64, P, P, P, P]
        L.hmxo_cg_dense.argtypes = [P, i64, i32, i32, f64, f64, P, P, f64, i32, P, P]
        L.hmxo_mlp_nparams.restype = C.c_int
        L.hmxo_mlp_forward.argtypes = [P, P, i64, P]
        L.hmxo_mlp_loss_grad.argtypes = [P, P, P, i64, f64, P, P]
        L.hmxo_mlp_adam.argtypes = [P, P, P, P, i64, i64, f64, f64, f64, f64]
        L.hmxo_features.argtypes = [P, P, P, P, i32, i64, i64, f64, P]
        L.hmxo_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def kind_of(kernel) -> int:
    return KINDS[kernel] if isinstance(kernel, str) else int(kernel)


def num_threads() -> int:
    return lib().hmxo_num_threads()


def kernel(kind, p0, x, y):
    x, y = _f64(x), _f64(y)
    return lib().hmxo_kernel(kind_of(kind), float(p0), _p(x), _p(y), int(x.shape[0]))


def xk1(s):
    """s K_1(s) (modified Bessel function of the second kind, order 1)."""
    return lib().hmxo_xk1(float(s))


def global_box(pts):
    pts = _f64(pts)
    n, d = pts.shape
    lo, hi = np.empty(d), np.empty(d)
    assert lib().hmxo_global_box(_p(pts), n, d, _p(lo), _p(hi)) == 0
    return lo, hi


def morton(pts, lo=None, hi=None):
    pts = _f64(pts)
    n, d = pts.shape
    if lo is None:
        lo, hi = global_box(pts)
    lo, hi = _f64(lo), _f64(hi)
    codes = np.empty(n, dtype=np.uint64)
    assert lib().hmxo_morton(_p(pts), n, d, _p(lo), _p(hi), _p(codes)) == 0
    return codes


def sort(codes):
    codes = np.ascontiguousarray(codes, dtype=np.uint64)
    perm = np.empty(codes.shape[0], dtype=np.int32)
    assert lib().hmxo_sort(_p(codes), codes.shape[0], _p(perm)) == 0
    return perm


def ordered_coords(pts, perm):
    pts = _f64(pts)
    n, d = pts.shape
    soa = np.empty((d, n))
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    lib().hmxo_ordered_coords(_p(pts), n, d, _p(perm), _p(soa))
    return soa


def order(pts):
    """Morton codes (original order), permutation, SoA ordered coordinates."""
    codes = morton(pts)
    perm = sort(codes)
    return codes, perm, ordered_coords(pts, perm)


def cluster_tree(n, leaf):
    cnt = lib().hmxo_cluster_tree(int(n), int(leaf), 0, None, None, None, None)
    lo = np.empty(cnt, np.int32)
    hi = np.empty(cnt, np.int32)
    dep = np.empty(cnt, np.int32)
    ch = np.empty(cnt, np.int64)
    assert lib().hmxo_cluster_tree(int(n), int(leaf), cnt, _p(lo), _p(hi), _p(dep), _p(ch)) == cnt
    return lo, hi, dep, ch


def boxes(soa, lo, hi):
    soa = _f64(soa)
    d, n = soa.shape
    lo = np.ascontiguousarray(lo, np.int32)
    hi = np.ascontiguousarray(hi, np.int32)
    nn = lo.shape[0]
    bmin = np.empty((nn, d))
    bmax = np.empty((nn, d))
    lib().hmxo_boxes(_p(soa), n, d, nn, _p(lo), _p(hi), _p(bmin), _p(bmax))
    return bmin, bmax


def admissible(amin, amax, bmin, bmax, eta):
    amin, amax, bmin, bmax = map(_f64, (amin, amax, bmin, bmax))
    return bool(lib().hmxo_admissible(_p(amin), _p(amax), _p(bmin), _p(bmax), amin.shape[0],
                                      float(eta)))


def partition(soa, leaf, eta):
    """Returns (adm, dense, level_sizes); leaves are int32 (k, 5) arrays of
    (tlo, thi, slo, shi, level) in canonical order."""
    soa = _f64(soa)
    d, n = soa.shape
    na, nd = C.c_int64(0), C.c_int64(0)
    ls = np.zeros(64, np.int64)
    nl = C.c_int32(0)
    cap_a = cap_d = 1024
    while True:
        adm = np.empty((cap_a, 5), np.int32)
        den = np.empty((cap_d, 5), np.int32)
        rc = lib().hmxo_partition(_p(soa), n, d, int(leaf), float(eta), cap_a, _p(adm),
                                  C.byref(na), cap_d, _p(den), C.byref(nd), _p(ls), C.byref(nl))
        if rc < 0:
            raise ValueError("hmxo_partition failed: %d" % rc)
        if rc == 0:
            return adm[: na.value].copy(), den[: nd.value].copy(), ls[: nl.value].copy()
        cap_a, cap_d = max(cap_a, na.value), max(cap_d, nd.value)


def aca(soa, kind, p0, tlo, thi, slo, shi, kmax, eps, aca_eta=0.0, eps0=1e-14, fixed=False,
        r_start=0, want_trace=False):
    """Algorithm 2 on one block: (U, V, rank, steps), plus the per-step trace
    (rank x 5: row pivot, column, row-pivot gap, stop-test ratio, next column
    gap) when want_trace."""
    soa = _f64(soa)
    d, n = soa.shape
    m, nc = thi - tlo, shi - slo
    U = np.zeros((kmax, m))
    V = np.zeros((kmax, nc))
    rk = C.c_int32(0)
    st = C.c_int32(0)
    tr = np.zeros((kmax, 5)) if want_trace else None
    rc = lib().hmxo_aca_traced(_p(soa), n, d, kind_of(kind), float(p0), tlo, thi, slo, shi,
                               int(kmax), float(eps), float(aca_eta), float(eps0),
                               int(bool(fixed)), int(r_start), _p(U), _p(V), C.byref(rk),
                               C.byref(st), _p(tr))
    assert rc == 0
    r = rk.value
    # stored column-major m x kmax == row-major (kmax, m)
    if want_trace:
        return U[:r].T.copy(), V[:r].T.copy(), r, st.value, tr[:r].copy()
    return U[:r].T.copy(), V[:r].T.copy(), r, st.value


def dense_block(soa, kind, p0, tlo, thi, slo, shi):
    soa = _f64(soa)
    d, n = soa.shape
    A = np.empty((shi - slo, thi - tlo))
    lib().hmxo_dense_block(_p(soa), n, d, kind_of(kind), float(p0), tlo, thi, slo, shi, _p(A))
    return A.T.copy()


def hmvp(pts, x, kind, p0, leaf, eta, kmax, eps, aca_eta=0.0, eps0=1e-14, fixed=False,
         sigma2=0.0, alpha=1.0, beta=0.0, z=None, want_ranks=False, symmetric=False):
    """z = alpha (H x + sigma2 x) + beta z; returns (z, ranks or None, stats dict).
    symmetric: only the admissible leaf with tau before sigma is approximated,
    its mirror applies the transposed factors."""
    pts = _f64(pts)
    n, d = pts.shape
    x = _f64(x)
    zz = _f64(z).copy() if z is not None else np.zeros(n)
    stats = np.zeros(8)
    cap = 0
    ranks = None
    if want_ranks:
        cap = 1 << 22
        ranks = np.zeros(cap, np.int32)
    rc = lib().hmxo_hmvp_ex(_p(pts), n, d, kind_of(kind), float(p0), int(leaf), float(eta),
                            int(kmax), float(eps), float(aca_eta), float(eps0), int(bool(fixed)),
                            int(bool(symmetric)), float(sigma2), float(alpha), float(beta), _p(x),
                            _p(zz), cap, _p(ranks), _p(stats))
    if rc != 0:
        raise ValueError("hmxo_hmvp failed: %d" % rc)
    st = dict(n_adm=int(stats[0]), n_dense=int(stats[1]), sum_rank=int(stats[2]),
              dense_entries=int(stats[3]), factor_entries=int(stats[4]), levels=int(stats[5]))
    if ranks is not None:
        ranks = ranks[: st["n_adm"]].copy()
    return zz, ranks, st


def dense_matvec(pts, x, kind, p0, sigma2=0.0, rows=None):
    """z = (A + sigma2 I) x (rows of z only, if given); x may be n x m."""
    pts = _f64(pts)
    n, d = pts.shape
    x = _f64(x)
    if x.ndim == 2:
        m = x.shape[1]
        r = None if rows is None else np.ascontiguousarray(rows, np.int64)
        cnt = n if r is None else r.shape[0]
        Z = np.empty((cnt, m))
        rc = lib().hmxo_dense_matmat(_p(pts), n, d, kind_of(kind), float(p0), float(sigma2),
                                     _p(x), m, None if r is None else _p(r), cnt, _p(Z))
        if rc != 0:
            raise ValueError("at most 64 right-hand sides")
        return Z
    if rows is None:
        z = np.empty(n)
        lib().hmxo_dense_matvec(_p(pts), n, d, kind_of(kind), float(p0), float(sigma2), _p(x),
                                None, 0, _p(z))
    else:
        rows = np.ascontiguousarray(rows, np.int64)
        z = np.empty(rows.shape[0])
        lib().hmxo_dense_matvec(_p(pts), n, d, kind_of(kind), float(p0), float(sigma2), _p(x),
                                _p(rows), rows.shape[0], _p(z))
    return z


def dense_matvec_rect(pts1, pts2, x, kind, p0):
    """z = A_{Y1 x Y2} x, the plain dense product (x: n2 entries, z: n1)."""
    pts1, pts2, x = _f64(pts1), _f64(pts2), _f64(x)
    n1, d = pts1.shape
    n2 = pts2.shape[0]
    z = np.empty(n1)
    lib().hmxo_dense_matvec_rect(_p(pts1), n1, _p(pts2), n2, d, kind_of(kind), float(p0), _p(x),
                                 _p(z))
    return z


def partition_rect(soa1, soa2, leaf, eta):
    """Leaves of A(Y1 x Y2) from the two sets' ordered coordinates: (adm,
    dense, level_sizes), rows in Y1's Morton order, columns in Y2's."""
    soa1, soa2 = _f64(soa1), _f64(soa2)
    d, n1 = soa1.shape
    n2 = soa2.shape[1]
    na, nd = C.c_int64(0), C.c_int64(0)
    ls = np.zeros(64, np.int64)
    nl = C.c_int32(0)
    cap_a = cap_d = 1024
    while True:
        adm = np.empty((cap_a, 5), np.int32)
        den = np.empty((cap_d, 5), np.int32)
        rc = lib().hmxo_partition_rect(_p(soa1), n1, _p(soa2), n2, d, int(leaf), float(eta),
                                       cap_a, _p(adm), C.byref(na), cap_d, _p(den), C.byref(nd),
                                       _p(ls), C.byref(nl))
        if rc < 0:
            raise ValueError("hmxo_partition_rect failed: %d" % rc)
        if rc == 0:
            return adm[: na.value].copy(), den[: nd.value].copy(), ls[: nl.value].copy()
        cap_a, cap_d = max(cap_a, na.value), max(cap_d, nd.value)


def hmvp_rect(pts1, pts2, x, kind, p0, leaf, eta, kmax, eps, aca_eta=0.0, eps0=1e-14,
              fixed=False, alpha=1.0, beta=0.0, z=None, want_ranks=False):
    """z = alpha H x + beta z for A(Y1 x Y2); returns (z, ranks or None, stats)."""
    pts1, pts2, x = _f64(pts1), _f64(pts2), _f64(x)
    n1, d = pts1.shape
    n2 = pts2.shape[0]
    zz = _f64(z).copy() if z is not None else np.zeros(n1)
    stats = np.zeros(8)
    cap = (1 << 22) if want_ranks else 0
    ranks = np.zeros(cap, np.int32) if want_ranks else None
    rc = lib().hmxo_hmvp_rect(_p(pts1), n1, _p(pts2), n2, d, kind_of(kind), float(p0), int(leaf),
                              float(eta), int(kmax), float(eps), float(aca_eta), float(eps0),
                              int(bool(fixed)), float(alpha), float(beta), _p(x), _p(zz), cap,
                              _p(ranks), _p(stats))
    if rc != 0:
        raise ValueError("hmxo_hmvp_rect failed: %d" % rc)
    st = dict(n_adm=int(stats[0]), n_dense=int(stats[1]), sum_rank=int(stats[2]),
              dense_entries=int(stats[3]), factor_entries=int(stats[4]), levels=int(stats[5]))
    if ranks is not None:
        ranks = ranks[: st["n_adm"]].copy()
    return zz, ranks, st


def hmvp_rows(pts, x, kind, p0, leaf, eta, kmax, eps, row_lo, row_hi, aca_eta=0.0, eps0=1e-14,
              fixed=False):
    """Stored-mode H x on Morton-order rows [row_lo, row_hi).  Returns
    (z_rows in Morton order, perm, dict of times / stored entries)."""
    pts = _f64(pts)
    n, d = pts.shape
    x = _f64(x)
    z = np.zeros(row_hi - row_lo)
    perm = np.empty(n, np.int32)
    t = np.zeros(5)
    rc = lib().hmxo_hmvp_rows(_p(pts), n, d, kind_of(kind), float(p0), int(leaf), float(eta),
                              int(kmax), float(eps), float(aca_eta), float(eps0), int(bool(fixed)),
                              int(row_lo), int(row_hi), _p(x), _p(z), _p(perm), _p(t))
    if rc != 0:
        raise ValueError("hmxo_hmvp_rows failed: %d" % rc)
    return z, perm, dict(partition_s=t[0], build_s=t[1], apply_s=t[2], entries=t[3],
                         blocks=int(t[4]))


def cg_dense(pts, b, kind, p0, sigma2, tol=1e-10, max_iter=10000):
    """CG on the dense (A + sigma2 I) x = b.  Returns (x, rc, iters, rel_res)."""
    pts = _f64(pts)
    n, d = pts.shape
    b = _f64(b)
    x = np.zeros(n)
    it, res = C.c_int32(0), C.c_double(0)
    rc = lib().hmxo_cg_dense(_p(pts), n, d, kind_of(kind), float(p0), float(sigma2), _p(b),
                             _p(x), float(tol), int(max_iter), C.byref(it), C.byref(res))
    return x, rc, it.value, res.value


def mlp_nparams():
    return lib().hmxo_mlp_nparams()


def mlp_forward(w, X):
    w, X = _f64(w), _f64(X)
    out = np.empty(X.shape[0])
    lib().hmxo_mlp_forward(_p(w), _p(X), X.shape[0], _p(out))
    return out


def mlp_loss_grad(w, X, y, q=0.9):
    w, X, y = _f64(w), _f64(X), _f64(y)
    g = np.empty(w.shape[0])
    loss = C.c_double(0)
    lib().hmxo_mlp_loss_grad(_p(w), _p(X), _p(y), X.shape[0], float(q), C.byref(loss), _p(g))
    return loss.value, g


def mlp_adam(w, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In place on float64 arrays w, m, v."""
    g = _f64(g)
    lib().hmxo_mlp_adam(_p(w), _p(m), _p(v), _p(g), w.shape[0], int(t), float(lr), float(b1),
                        float(b2), float(eps))


def features(ta, tb, sa, sb, m, n, ell):
    ta, tb, sa, sb = map(_f64, (ta, tb, sa, sb))
    f = np.empty(8)
    lib().hmxo_features(_p(ta), _p(tb), _p(sa), _p(sb), ta.shape[0], int(m), int(n), float(ell),
                        _p(f))
    return f
