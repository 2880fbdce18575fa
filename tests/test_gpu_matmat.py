"""The product with several right-hand sides (hmx_matmat): each column of
Z = alpha (H + sigma2 I) X + beta Z equals the single-vector product of the
matching column of X to rounding (the same stored entries and weights,
summed in another order), for every storage mode, the symmetric far field,
the recomputed near field and rectangular handles; in FP64 it also meets
the oracle's dense product for many right-hand sides."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_09707_amd import hmx
    hmx.lib()
    return hmx


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _columns(H, hm, X, Z0, alpha, beta):
    """The single-vector products, one column at a time."""
    out = []
    for c in range(X.shape[0]):
        z = Z0[c].clone()
        H.hmx_matvec(hm.h, X[c].contiguous(), z, alpha, beta)
        out.append(z)
    return torch.stack(out)


MODES = [  # compute, storage, near, symmetric, near_recompute, tolerance
    ("f64", "f64", "f64", 0, 0, 1e-13),
    ("f64", "f64", "f64", 1, 1, 1e-13),
    ("f32", "f32", "f32", 0, 0, 2e-6),
    ("f32", "bf16", "bf16", 1, 0, 2e-6),
    ("f32", "bf16", "f32", 0, 0, 2e-6),
    ("f32", "bf16", "bf16", 0, 1, 2e-6),
]


@pytest.mark.parametrize("mode", MODES)
def test_matmat_columns_equal_matvec(H, mode):
    cd, sd, nd, sym, nr, tol = mode
    n, m = 12000, 37  # 37 = 16 + 16 + 4 + 1 right-hand sides
    dt = np.float64 if cd == "f64" else np.float32
    pts = synth.uniform_points(n, 3, 700, dtype=dt)
    print("build: N=%d d=3 %s/%s/%s sym=%d near_recompute=%d, %d right-hand sides"
          % (n, cd, sd, nd, sym, nr, m), flush=True)
    hm = H.HMatrix(_dev(pts), "gaussian", 0.05, compute_dtype=cd, storage_dtype=sd,
                   near_dtype=nd, symmetric_far=sym, near_recompute=nr, leaf_size=64, eta=1.5,
                   aca_eps=1e-6, max_rank=48, sigma2=0.3)
    g = synth.rng(701)
    X = _dev(g.standard_normal((m, n)).astype(dt))
    Z0 = _dev(g.standard_normal((m, n)).astype(dt))
    Z = Z0.clone()
    H.hmx_matmat(hm.h, X, Z, 0.75, -1.5)
    ref = _columns(H, hm, X, Z0, 0.75, -1.5)
    e = _rel(Z.double().cpu().numpy(), ref.double().cpu().numpy())
    worst = max(_rel(Z[c].double().cpu().numpy(), ref[c].double().cpu().numpy())
                for c in range(m))
    print("  matmat vs column-wise matvec: %.2e (worst column %.2e)" % (e, worst), flush=True)
    assert worst <= tol
    # the work vectors are kept: a second call (another m) allocates nothing new
    b = hm.stats().device_bytes
    Z2 = hm.matmat(X[:3])
    assert hm.stats().device_bytes == b
    assert _rel(Z2.double().cpu().numpy(), _columns(H, hm, X[:3], torch.zeros_like(Z0[:3]),
                                                     1.0, 0.0).double().cpu().numpy()) <= tol
    hm.close()


def test_matmat_f64_against_oracle_dense(H, orc):
    n, m, eps = 4096, 16, 1e-8
    pts = synth.uniform_points(n, 2, 710)
    g = synth.rng(711)
    Xh = g.standard_normal((m, n))
    hm = H.HMatrix(_dev(pts), "matern32", 0.1, compute_dtype="f64", leaf_size=64, eta=1.5,
                   aca_eps=eps, max_rank=64)
    Z = hm.matmat(_dev(Xh)).cpu().numpy()
    Zd = orc.dense_matvec(pts, np.ascontiguousarray(Xh.T), "matern32", 0.1).T
    e = _rel(Z, Zd)
    print("matmat (16 sides) vs oracle dense product: %.2e" % e, flush=True)
    assert e <= 10 * eps
    hm.close()


def test_matmat_rect_with_leading_dimensions(H, orc):
    n1, n2, m = 7000, 3000, 9  # 8 + 1
    p1 = synth.uniform_points(n1, 2, 720)
    p2 = synth.uniform_points(n2, 2, 721) * 1.2 + 0.4
    g = synth.rng(722)
    Xp = g.standard_normal((m, n2 + 5))  # leading dimension n2 + 5: padding ignored
    Zp = g.standard_normal((m, n1 + 3))
    hm = H.HMatrix.rect(_dev(p1), _dev(p2), "gaussian", 0.02, compute_dtype="f64",
                        leaf_size=64, eta=1.5, aca_eps=1e-8, max_rank=48)
    X, Z = _dev(Xp), _dev(Zp)
    H.hmx_matmat(hm.h, X, Z, 2.0, 0.5)
    Zh = Z.cpu().numpy()
    assert np.array_equal(Zh[:, n1:], Zp[:, n1:])  # past each column: untouched
    for c in range(m):
        zo, _, _ = orc.hmvp_rect(p1, p2, Xp[c, :n2], "gaussian", 0.02, 64, 1.5, 48, 1e-8)
        ref = 2.0 * zo + 0.5 * Zp[c, :n1]
        assert _rel(Zh[c, :n1], ref) <= 1e-12, c
    with pytest.raises(ValueError):
        H.hmx_matmat(hm.h, _dev(Xp[:, :n2 - 1]), Z)
    hm.close()


def test_matmat_refusals(H):
    pts = _dev(synth.uniform_points(2000, 2, 730))
    hn = H.HMatrix(pts, "gaussian", 0.05, compute_dtype="f64", far_recompute=1)
    X = torch.zeros((2, 2000), dtype=torch.float64, device="cuda:0")
    with pytest.raises(H.HmxError) as e:
        H.hmx_matmat(hn.h, X, torch.zeros_like(X))
    assert e.value.status == H.HMX_ERR_UNSUPPORTED
    hn.close()
    hs = H.HMatrix(pts, "gaussian", 0.05, compute_dtype="f64")
    with pytest.raises(H.HmxError) as e:  # m = 0
        H.hmx_matmat(hs.h, X[:0], X[:0].clone())
    assert e.value.status == H.HMX_ERR_INVALID_ARG
    with pytest.raises(H.HmxError):  # dtype must be the compute dtype
        H.hmx_matmat(hs.h, X.float(), X.float().clone())
    hs.close()


# Two summation orders of K terms differ by about sqrt(K) u relative to the
# result (random signs); a 600-point tile sums about 10^4 columns per row,
# so FP32 (u = 2^-24) allows 8 sqrt(10^4) u = 5e-6 there, 2e-6 on 256-point
# tiles (about 3 10^3 columns).
WIDE = [  # compute, storage, near, leaf: 256-row tiles (four waves per workgroup), 600-row
    # tiles (row passes, phase 1 reading X from the vector), ragged tile sizes
    ("f64", "f64", "f64", 256, 1e-13),
    ("f32", "f32", "f32", 256, 2e-6),
    ("f32", "bf16", "bf16", 256, 2e-6),
    ("f32", "bf16", "f32", 256, 2e-6),
    ("f64", "f64", "f64", 600, 1e-13),
    ("f32", "bf16", "bf16", 600, 5e-6),
]


@pytest.mark.parametrize("mode", WIDE)
def test_matmat_wide_tiles_matrix_cores(H, mode):
    """The matrix-core forms (8 and 16 sides) on tiles of 150-256 and 300-600
    rows: every column equals the single-vector product to rounding."""
    cd, sd, nd, leaf, tol = mode
    n, m = 45000, 24  # 16 + 8 sides; N not a power of two: tile sizes differ
    dt = np.float64 if cd == "f64" else np.float32
    pts = synth.uniform_points(n, 2, 740, dtype=dt)
    print("build: N=%d d=2 %s/%s/%s leaf %d, %d right-hand sides" % (n, cd, sd, nd, leaf, m),
          flush=True)
    hm = H.HMatrix(_dev(pts), "gaussian", 0.02, compute_dtype=cd, storage_dtype=sd,
                   near_dtype=nd, leaf_size=leaf, eta=1.5, aca_eps=1e-6, max_rank=32, sigma2=0.1)
    g = synth.rng(741)
    X = _dev(g.standard_normal((m, n)).astype(dt))
    Z0 = _dev(g.standard_normal((m, n)).astype(dt))
    Z = Z0.clone()
    H.hmx_matmat(hm.h, X, Z, 1.25, 0.5)
    ref = _columns(H, hm, X, Z0, 1.25, 0.5)
    worst = max(_rel(Z[c].double().cpu().numpy(), ref[c].double().cpu().numpy())
                for c in range(m))
    print("  worst column vs matvec: %.2e" % worst, flush=True)
    assert worst <= tol
    hm.close()


@pytest.mark.parametrize("sd", ["f32", "bf16", "f64"])
def test_matmat_padded_groups(H, sd):
    """Groups of 3, 5, 13 and 17 sides (the rest of 16 padded with zero sides on
    the matrix cores, a last single side as a matvec): every column equals the
    single-vector product to rounding, and memory past Z's m columns is never
    written."""
    cd = "f64" if sd == "f64" else "f32"
    dt = np.float64 if cd == "f64" else np.float32
    tol = 1e-13 if cd == "f64" else 2e-6
    n = 20000
    pts = synth.uniform_points(n, 2, 750, dtype=dt)
    hm = H.HMatrix(_dev(pts), "gaussian", 0.02, compute_dtype=cd, storage_dtype=sd,
                   leaf_size=256, eta=1.5, aca_eps=1e-6, max_rank=32, sigma2=0.2)
    g = synth.rng(751)
    for m in (3, 5, 13, 17):
        print("storage %s, %d sides" % (sd, m), flush=True)
        X = _dev(g.standard_normal((m, n)).astype(dt))
        Zall = _dev(g.standard_normal((m + 2, n)).astype(dt))
        before = Zall.clone()
        Z = Zall[:m]
        H.hmx_matmat(hm.h, X, Z, 0.5, 2.0)
        assert torch.equal(Zall[m:], before[m:]), "rows past the m sides were written"
        ref = _columns(H, hm, X, before[:m], 0.5, 2.0)
        worst = max(_rel(Z[c].double().cpu().numpy(), ref[c].double().cpu().numpy())
                    for c in range(m))
        assert worst <= tol, (m, worst)
    hm.close()
