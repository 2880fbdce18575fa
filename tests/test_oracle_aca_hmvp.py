"""Pins for the oracle's kernel functions, ACA (Algorithm 2) and H-matrix-vector
product (Algorithm 3).  CPU only."""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

import synth


def _dense(pts, kind, p0):
    r = cdist(pts, pts)
    if kind == "gaussian":
        return np.exp(-(r ** 2) / p0)
    if kind == "matern32":
        s = np.sqrt(3.0) * r / p0
        return (1 + s) * np.exp(-s)
    if kind == "const":
        return np.ones_like(r)
    if kind == "lowrank":
        return (1.0 + pts @ pts.T) ** 2
    raise ValueError(kind)


@pytest.mark.parametrize("kind,p0", [("gaussian", 0.1), ("matern32", 0.3), ("const", 1.0),
                                     ("lowrank", 1.0)])
def test_dense_matvec_matches_scipy(orc, kind, p0):
    p = synth.uniform_points(700, 3, 1)
    x = synth.normal_vector(700, 2)
    want = _dense(p, kind, p0) @ x + 0.5 * x
    got = orc.dense_matvec(p, x, kind, p0, sigma2=0.5)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())
    rows = np.array([0, 5, 699])
    assert np.allclose(orc.dense_matvec(p, x, kind, p0, sigma2=0.5, rows=rows), want[rows],
                       rtol=1e-12, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("kind,p0", [("gaussian", 0.1), ("matern_nu1", 0.2)])
def test_dense_matmat_columns_equal_matvec(orc, kind, p0):
    """The multi-right-hand-side dense product sums every column as the
    single-vector one does: equal bit for bit, with rows and the shift."""
    p = synth.uniform_points(500, 2, 7)
    X = np.stack([synth.normal_vector(500, 20 + c) for c in range(5)], axis=1)
    Z = orc.dense_matvec(p, X, kind, p0, sigma2=0.25)
    rows = np.array([3, 0, 499])
    Zr = orc.dense_matvec(p, X, kind, p0, sigma2=0.25, rows=rows)
    for c in range(5):
        z = orc.dense_matvec(p, X[:, c], kind, p0, sigma2=0.25)
        assert np.array_equal(Z[:, c], z)
        assert np.array_equal(Zr[:, c], z[rows])
    want = _dense(p, "gaussian", p0) @ X if kind == "gaussian" else None
    if want is not None:
        assert np.allclose(Z - 0.25 * X, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


def _block(seed=3, n=2000, d=2, leaf=64, eta=1.5, pick=-1):
    p = synth.uniform_points(n, d, seed)
    _, _, soa = __import__("oracle").order(p)
    adm, den, _ = __import__("oracle").partition(soa, leaf, eta)
    return soa, adm[pick]


def test_aca_const_kernel_rank_one(orc):
    soa, b = _block()
    U, V, r, steps = orc.aca(soa, "const", 1.0, b[0], b[1], b[2], b[3], 16, 1e-8)
    assert r == 1
    A = orc.dense_block(soa, "const", 1.0, *b[:4])
    assert np.abs(A - U @ V.T).max() <= 1e-14
    # the eps0 guard rejects every further column; kmax failed columns end it
    assert steps == 1 + 16


@pytest.mark.parametrize("d,maxrank", [(2, 6), (3, 10)])
def test_aca_lowrank_kernel_exact(orc, d, maxrank):
    soa, b = _block(d=d, n=3000)
    U, V, r, _ = orc.aca(soa, "lowrank", 1.0, b[0], b[1], b[2], b[3], 32, 0.0, eps0=1e-10)
    assert r <= maxrank
    A = orc.dense_block(soa, "lowrank", 1.0, *b[:4])
    assert np.linalg.norm(A - U @ V.T) <= 1e-12 * np.linalg.norm(A)
    assert r == np.linalg.matrix_rank(A)


@pytest.mark.parametrize("eps", [1e-3, 1e-6, 1e-9])
def test_aca_gaussian_error_bound_and_svd_floor(orc, eps):
    soa, _ = _block()
    p = synth.uniform_points(2000, 2, 3)
    _, _, soa = orc.order(p)
    adm, _, _ = orc.partition(soa, 64, 1.5)
    rng = np.random.default_rng(0)
    for q in rng.choice(len(adm), 12, replace=False):
        b = adm[q]
        U, V, r, _ = orc.aca(soa, "gaussian", 0.1, b[0], b[1], b[2], b[3], 64, eps)
        A = orc.dense_block(soa, "gaussian", 0.1, *b[:4])
        err = np.linalg.norm(A - U @ V.T)
        assert err <= 10 * eps * np.linalg.norm(A) + 1e-13
        s = np.linalg.svd(A, compute_uv=False)
        assert err >= np.sqrt((s[r:] ** 2).sum()) * (1 - 1e-8) - 1e-14  # Eckart-Young floor


def test_aca_full_rank_is_exact(orc):
    soa, b = _block(n=600, leaf=16, pick=0)
    m, n = b[1] - b[0], b[3] - b[2]
    U, V, r, _ = orc.aca(soa, "gaussian", 0.1, b[0], b[1], b[2], b[3], min(m, n), 0.0, eps0=0.0)
    A = orc.dense_block(soa, "gaussian", 0.1, *b[:4])
    assert r == min(m, n)
    assert np.linalg.norm(A - U @ V.T) <= 1e-10 * np.linalg.norm(A)


def test_aca_pivot_structure(orc):
    """u_r is normalised at its pivot row; the residual vanishes on pivot rows."""
    soa, b = _block(n=2000, pick=5)
    U, V, r, _ = orc.aca(soa, "gaussian", 0.1, b[0], b[1], b[2], b[3], 20, 0.0, fixed=True)
    assert r == 20
    A = orc.dense_block(soa, "gaussian", 0.1, *b[:4])
    piv_rows = [int(np.argmax(np.abs(U[:, l]) == 1.0)) for l in range(r)]
    assert len(set(piv_rows)) == r
    for l, i in enumerate(piv_rows):
        assert U[i, l] == 1.0
        assert np.all(U[i, l + 1:] == 0.0) or np.abs(U[i, l + 1:]).max() < 1e-12
    R = A - U @ V.T
    assert np.abs(R[piv_rows, :]).max() <= 1e-12 * np.abs(A).max()
    # the first column pivot is the sigma point nearest to tau's box centre
    c = 0.5 * (soa[:, b[0]:b[1]].min(1) + soa[:, b[0]:b[1]].max(1))
    j1 = int(np.argmin(((soa[:, b[2]:b[3]] - c[:, None]) ** 2).sum(0)))
    assert np.abs(R[:, j1]).max() <= 1e-12 * np.abs(A).max()
    assert np.abs(U[:, 0] * V[j1, 0] - A[:, j1]).max() <= 1e-12 * np.abs(A).max()


def test_aca_fixed_and_one_shot(orc):
    soa, b = _block(n=2000, pick=3)
    args = (soa, "gaussian", 0.1, b[0], b[1], b[2], b[3], 40)
    U1, V1, r1, _ = orc.aca(*args, 1e-6)
    # one-shot started below the adaptive rank continues to the same factors
    U2, V2, r2, _ = orc.aca(*args, 1e-6, r_start=max(1, r1 - 3))
    assert r2 == r1 and np.array_equal(U1, U2) and np.array_equal(V1, V2)
    # one-shot at the adaptive rank passes its final check
    U3, V3, r3, _ = orc.aca(*args, 1e-6, r_start=r1)
    assert r3 == r1 and np.array_equal(U1, U3)
    # one-shot above it keeps the extra terms (at least as accurate)
    U4, V4, r4, _ = orc.aca(*args, 1e-6, r_start=r1 + 4)
    assert r4 == r1 + 4 and np.array_equal(U4[:, :r1], U1)
    # fixed rank ignores the stopping test
    U5, V5, r5, _ = orc.aca(*args, 1e-2, fixed=True)
    assert r5 == 40


def test_hmvp_eta_zero_is_dense(orc):
    p = synth.uniform_points(1500, 2, 4)
    x = synth.normal_vector(1500, 5)
    z, _, st = orc.hmvp(p, x, "gaussian", 0.1, 32, 0.0, 16, 1e-3)
    assert st["n_adm"] == 0
    zd = _dense(p, "gaussian", 0.1) @ x
    assert np.linalg.norm(z - zd) <= 1e-13 * np.linalg.norm(zd)


def test_hmvp_leaf_ge_n_is_dense(orc):
    p = synth.uniform_points(500, 3, 4)
    x = synth.normal_vector(500, 5)
    z, _, st = orc.hmvp(p, x, "matern32", 0.2, 500, 1.5, 16, 1e-3)
    assert st["n_adm"] == 0 and st["n_dense"] == 1
    zd = _dense(p, "matern32", 0.2) @ x
    assert np.linalg.norm(z - zd) <= 1e-13 * np.linalg.norm(zd)


def test_hmvp_const_kernel_closed_form(orc):
    p = synth.uniform_points(3000, 2, 6)
    x = synth.normal_vector(3000, 7)
    z, ranks, st = orc.hmvp(p, x, "const", 1.0, 64, 1.5, 8, 1e-8, sigma2=0.25, want_ranks=True)
    assert st["n_adm"] > 0 and np.all(ranks == 1)
    assert np.allclose(z, x.sum() + 0.25 * x, rtol=0, atol=1e-11)


def test_hmvp_exact_when_aca_is_exact(orc):
    p = synth.uniform_points(1200, 2, 8)
    x = synth.normal_vector(1200, 9)
    z, _, st = orc.hmvp(p, x, "gaussian", 0.1, 32, 1.5, 600, 0.0, eps0=0.0)
    zd = _dense(p, "gaussian", 0.1) @ x
    assert st["n_adm"] > 0
    assert np.linalg.norm(z - zd) <= 1e-11 * np.linalg.norm(zd)


def test_hmvp_small_workload_error(orc):
    """The small FP64 workload (N=4096, 2-d, Gaussian p0=0.1, leaf 64, eta 1.5,
    eps 1e-6, kmax 32) meets e_rel <= 10 eps against the dense product."""
    p = synth.uniform_points(4096, 2, 11)
    x = synth.normal_vector(4096, 12)
    z, _, st = orc.hmvp(p, x, "gaussian", 0.1, 64, 1.5, 32, 1e-6)
    zd = _dense(p, "gaussian", 0.1) @ x
    err = np.linalg.norm(z - zd) / np.linalg.norm(zd)
    assert err <= 1e-5


def test_hmvp_error_decreases_with_eps(orc):
    p = synth.uniform_points(3000, 3, 13)
    x = synth.normal_vector(3000, 14)
    zd = _dense(p, "gaussian", 0.05) @ x
    errs = []
    for eps in [1e-2, 1e-4, 1e-6, 1e-8]:
        z, _, _ = orc.hmvp(p, x, "gaussian", 0.05, 64, 1.5, 64, eps)
        errs.append(np.linalg.norm(z - zd) / np.linalg.norm(zd))
    assert all(errs[i + 1] < errs[i] for i in range(3)), errs
    assert errs[-1] < 1e-7


def test_hmvp_alpha_beta_sigma(orc):
    p = synth.uniform_points(800, 2, 15)
    x = synth.normal_vector(800, 16)
    z0 = synth.normal_vector(800, 17)
    base, _, _ = orc.hmvp(p, x, "gaussian", 0.1, 32, 1.5, 16, 1e-8)
    z, _, _ = orc.hmvp(p, x, "gaussian", 0.1, 32, 1.5, 16, 1e-8, sigma2=0.3, alpha=2.0,
                       beta=-0.5, z=z0)
    assert np.allclose(z, 2.0 * (base + 0.3 * x) - 0.5 * z0, rtol=1e-13, atol=1e-13)


def test_aca_stops_at_first_rank_meeting_the_criterion(orc):
    """The stopping rule of Algorithm 2 evaluated independently with numpy on
    the returned factors: |u_l| |v_l| <= eps/(1+eps) |sum_{k<=l} u_k v_k^T|_F
    fails for every l < r and holds at l = r."""
    p = synth.uniform_points(3000, 2, 21)
    _, _, soa = orc.order(p)
    adm, _, _ = orc.partition(soa, 64, 1.5)
    rng = np.random.default_rng(1)
    eps = 1e-5
    checked = 0
    for q in rng.choice(len(adm), 10, replace=False):
        b = adm[q]
        U, V, r, steps = orc.aca(soa, "gaussian", 0.05, b[0], b[1], b[2], b[3], 64, eps)
        if r == 64 or steps != r:
            continue
        for l in range(1, r + 1):
            lhs = np.linalg.norm(U[:, l - 1]) * np.linalg.norm(V[:, l - 1])
            rhs = eps / (1 + eps) * np.linalg.norm(U[:, :l] @ V[:, :l].T)
            assert (lhs <= rhs) == (l == r), (q, l, r, lhs, rhs)
        checked += 1
    assert checked >= 5


def test_cg_dense_matches_cholesky(orc):
    """The oracle's CG on (A + sigma2 I) c = y (kernel ridge regression) agrees
    with a dense Cholesky solve; it stops at the requested recurrence residual
    and its true residual is of the same size."""
    from scipy.linalg import cho_factor, cho_solve
    pts = synth.gmm_points(600, 3, 31, ncomp=8)
    y = synth.krr_target(pts, 32)
    A = _dense(pts, "matern32", 0.1) + 1e-2 * np.eye(600)
    c_ref = cho_solve(cho_factor(A), y)
    c, rc, it, res = orc.cg_dense(pts, y, "matern32", 0.1, 1e-2, tol=1e-10)
    assert rc == 0 and res <= 1e-10 and it < 600
    assert np.linalg.norm(c - c_ref) <= 1e-6 * np.linalg.norm(c_ref)
    assert np.linalg.norm(A @ c - y) <= 1e-9 * np.linalg.norm(y)
    # max_iter = 1: not converged, one iteration; b = 0: converged at once
    _, rc1, it1, _ = orc.cg_dense(pts, y, "matern32", 0.1, 1e-2, tol=1e-10, max_iter=1)
    assert rc1 == 1 and it1 == 1
    x0, rc0, it0, _ = orc.cg_dense(pts, np.zeros(600), "matern32", 0.1, 1e-2)
    assert rc0 == 0 and it0 == 0 and not x0.any()


@pytest.mark.parametrize("lo,hi", [(0, 1500), (0, 1), (700, 701), (333, 1111), (1499, 1500),
                                   (64, 128), (37, 1300)])
def test_hmvp_rows_equals_full_hmvp_slice(orc, lo, hi):
    """The row-range form of the H-matrix-vector product (Algorithm 3
    restricted to Morton rows [lo, hi), every block meeting the range built
    by Algorithm 2 and applied once) equals the Morton-ordered slice of the
    full product; ranges that cut through leaf clusters included.  The full
    product itself is pinned to the dense product above, and the slice is
    checked against the dense rows here as well."""
    n, leaf, eps = 1500, 32, 1e-7
    p = synth.uniform_points(n, 2, 101)
    x = synth.normal_vector(n, 102)
    z_full, _, _ = orc.hmvp(p, x, "gaussian", 0.05, leaf, 1.5, 48, eps)
    codes, perm, _ = orc.order(p)
    zr, perm_r, info = orc.hmvp_rows(p, x, "gaussian", 0.05, leaf, 1.5, 48, eps, lo, hi)
    assert np.array_equal(perm_r, perm)
    want = z_full[perm[lo:hi]]
    assert zr.shape == (hi - lo,)
    assert np.max(np.abs(zr - want)) <= 1e-14 * max(1.0, np.max(np.abs(want)))
    zd = orc.dense_matvec(p, x, "gaussian", 0.05, rows=perm[lo:hi])
    assert np.linalg.norm(zr - zd) <= 10 * eps * np.linalg.norm(zd) + 1e-14
    assert info["blocks"] > 0 and info["entries"] > 0


def test_hmvp_rows_invalid_ranges(orc):
    p = synth.uniform_points(100, 2, 103)
    x = synth.normal_vector(100, 104)
    for lo, hi in [(5, 5), (-1, 10), (0, 101), (50, 20)]:
        with pytest.raises(ValueError):
            orc.hmvp_rows(p, x, "gaussian", 0.05, 16, 1.5, 16, 1e-6, lo, hi)


def test_aca_trace_describes_the_run(orc):
    """The traced ACA returns the same factors as the plain call, and its
    trace is consistent with them: u_r is 1 at its pivot row, the stop-test
    ratio exceeds 1 before the last step and not at it, and every recorded
    gap lies in [0, 1]."""
    p = synth.uniform_points(2000, 2, 31)
    _, _, soa = orc.order(p)
    adm, _, _ = orc.partition(soa, 64, 1.5)
    b = adm[len(adm) // 3]
    U0, V0, r0, s0 = orc.aca(soa, "gaussian", 0.05, *b[:4], 32, 1e-6)
    U, V, r, s, tr = orc.aca(soa, "gaussian", 0.05, *b[:4], 32, 1e-6, want_trace=True)
    assert r == r0 and s == s0 and np.array_equal(U, U0) and np.array_equal(V, V0)
    assert r >= 3
    for q in range(r):
        assert U[int(tr[q, 0]), q] == 1.0
    assert np.all(tr[: r - 1, 3] > 1.0) and tr[r - 1, 3] <= 1.0
    assert np.all((tr[:, 2] >= 0) & (tr[:, 2] <= 1)) and np.all((tr[:, 4] >= 0) & (tr[:, 4] <= 1))
    assert len(set(tr[:, 1].astype(int))) == r  # distinct columns


def test_symmetric_far_field_oracle(orc):
    """The symmetric far field: each admissible leaf with tau before sigma is
    approximated once and its mirror (sigma, tau) applies V U^T.  Pinned by
    (a) exact symmetry of the operator, which the two-sided form lacks,
    (b) an independent assembly of the dense H from the leaves (ACA of the
    primary leaves, transposed at their mirrors, dense leaves entry by
    entry), (c) the error bound against the dense product, (d) the ranks:
    a mirror carries its primary's rank and a primary's rank is the
    two-sided run's, (e) exact ACA reducing it to the dense product."""
    n, leaf, eta, kmax, eps, p0 = 1500, 32, 1.5, 32, 1e-7, 0.05
    p = synth.uniform_points(n, 2, 4401)
    x = synth.normal_vector(n, 4402)
    y = synth.normal_vector(n, 4403)
    kw = dict(want_ranks=True)
    zx, rs, st = orc.hmvp(p, x, "gaussian", p0, leaf, eta, kmax, eps, symmetric=True, **kw)
    zy, _, _ = orc.hmvp(p, y, "gaussian", p0, leaf, eta, kmax, eps, symmetric=True)
    zx2, r2, st2 = orc.hmvp(p, x, "gaussian", p0, leaf, eta, kmax, eps, **kw)
    zy2, _, _ = orc.hmvp(p, y, "gaussian", p0, leaf, eta, kmax, eps)
    asym = abs(y @ zx - x @ zy) / (np.linalg.norm(y) * np.linalg.norm(zx))
    asym2 = abs(y @ zx2 - x @ zy2) / (np.linalg.norm(y) * np.linalg.norm(zx2))
    assert asym <= 1e-14 and asym2 > 100 * asym, (asym, asym2)
    # (b) assembly of the dense H in Morton order from the leaves
    _, perm, soa = orc.order(p)
    adm, den, _ = orc.partition(soa, leaf, eta)
    Hm = np.zeros((n, n))
    for b in den:
        Hm[b[0]:b[1], b[2]:b[3]] = orc.dense_block(soa, "gaussian", p0, *b[:4])
    for b in adm:
        if b[0] > b[2]:
            continue
        U, V, r, _ = orc.aca(soa, "gaussian", p0, *b[:4], kmax, eps)
        Hm[b[0]:b[1], b[2]:b[3]] = U @ V.T
        Hm[b[2]:b[3], b[0]:b[1]] = (U @ V.T).T
    zm = np.empty(n)
    zm[perm] = Hm @ x[perm]
    assert np.linalg.norm(zm - zx) <= 1e-13 * np.linalg.norm(zx)
    # (c) the bound of the two-sided form
    zd = orc.dense_matvec(p, x, "gaussian", p0)
    assert np.linalg.norm(zx - zd) <= 10 * eps * np.linalg.norm(zd)
    # (d) ranks: mirrors carry their primary's, primaries the two-sided run's
    key = {(int(b[0]), int(b[2])): q for q, b in enumerate(adm)}
    prim = adm[:, 0] <= adm[:, 2]
    assert np.array_equal(rs[prim], r2[prim])
    for q, b in enumerate(adm):
        if b[0] > b[2]:
            assert rs[q] == rs[key[(int(b[2]), int(b[0]))]]
    assert st["sum_rank"] == rs.sum() and st["factor_entries"] < st2["factor_entries"]
    # (e) exact ACA: the dense product
    q = synth.uniform_points(600, 2, 4404)
    xq = synth.normal_vector(600, 4405)
    ze, _, _ = orc.hmvp(q, xq, "gaussian", p0, 16, eta, 128, 0.0, eps0=0.0, symmetric=True)
    zdq = orc.dense_matvec(q, xq, "gaussian", p0)
    assert np.linalg.norm(ze - zdq) <= 1e-12 * np.linalg.norm(zdq)
