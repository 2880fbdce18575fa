"""The far field without precomputation (far_recompute: the paper's default
mode, Section 5.4; chunks of the ACA list within a bs_ACA-like budget,
Section 5.4.1).

Every product runs the same ACA as a stored build (Algorithm 2, same pivots
and tests), so after a matvec the ranks equal the stored build's bit for
bit; the far-field sums run per chunk in another order, so the products
agree to rounding: FP64 within 1e-13 relative, FP32 within 2e-6.  The FP64
product is also compared with the oracle's H-matrix-vector product (the same
approximation; the paper decides both) and its dense product.
"""
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


def _pair(H, pts, kern, p0, **kw):
    """A stored handle and a far_recompute handle with the same parameters."""
    hs = H.HMatrix(_dev(pts), kern, p0, **kw)
    hn = H.HMatrix(_dev(pts), kern, p0, far_recompute=1, **kw)
    return hs, hn


@pytest.mark.parametrize("near_recompute", [0, 1])
def test_np_f64_equals_stored_and_oracle(H, orc, near_recompute):
    n, p0, leaf, eta, eps, kmax = 4096, 0.1, 64, 1.5, 1e-6, 32
    pts = synth.uniform_points(n, 2, 11)
    x = synth.normal_vector(n, 12)
    print("build: N=%d d=2 gaussian F64 far_recompute near_recompute=%d" % (n, near_recompute),
          flush=True)
    hs, hn = _pair(H, pts, "gaussian", p0, compute_dtype="f64", leaf_size=leaf, eta=eta,
                   aca_eps=eps, max_rank=kmax, near_recompute=near_recompute)
    assert not hn.ranks().any()  # no ACA at build time
    st = hn.stats()
    assert st.n_adm == hs.stats().n_adm and st.aca_chunks == 1
    assert st.device_bytes < hs.stats().device_bytes
    zs = hs.matvec(_dev(x)).cpu().numpy()
    zn = hn.matvec(_dev(x)).cpu().numpy()
    assert np.array_equal(hn.ranks(), hs.ranks())
    assert hn.stats().sum_rank == hs.stats().sum_rank
    e_s = _rel(zn, zs)
    zo, ranks_o, _ = orc.hmvp(pts, x, "gaussian", p0, leaf, eta, kmax, eps, want_ranks=True)
    zd = orc.dense_matvec(pts, x, "gaussian", p0)
    e_o, e_d = _rel(zn, zo), _rel(zn, zd)
    print("  NP vs stored %.2e, vs oracle H %.2e, vs dense %.2e" % (e_s, e_o, e_d), flush=True)
    assert e_s <= 1e-13
    assert e_d <= 10 * eps
    # the oracle's ranks may differ from the GPU's at pivot near-ties only
    # (covered by the parity tests); the products agree to the ACA tolerance
    assert e_o <= 10 * eps
    # a second product repeats the first bit for bit
    assert np.array_equal(hn.matvec(_dev(x)).cpu().numpy(), zn)
    hs.close()
    hn.close()


def test_np_many_chunks_equal_one_chunk(H):
    """A 1 MiB budget cuts the list into many chunks (each a share of every
    level); ranks are those of the single chunk bit for bit, products agree
    to rounding."""
    n, p0 = 6000, 0.05
    pts = synth.uniform_points(n, 3, 21)
    x = synth.normal_vector(n, 22)
    kw = dict(compute_dtype="f64", leaf_size=48, eta=1.5, aca_eps=1e-7, max_rank=40,
              far_recompute=1)
    print("build: N=%d d=3 F64 far_recompute, one chunk and a 1 MiB budget" % n, flush=True)
    h1 = H.HMatrix(_dev(pts), "gaussian", p0, **kw)
    hm = H.HMatrix(_dev(pts), "gaussian", p0, aca_chunk_mb=1, **kw)
    assert h1.stats().aca_chunks == 1
    nch = hm.stats().aca_chunks
    print("  chunks: %d" % nch, flush=True)
    assert nch > 8
    z1 = h1.matvec(_dev(x)).cpu().numpy()
    zm = hm.matvec(_dev(x)).cpu().numpy()
    assert np.array_equal(h1.ranks(), hm.ranks())
    e = _rel(zm, z1)
    print("  many chunks vs one: %.2e" % e, flush=True)
    assert e <= 1e-13
    h1.close()
    hm.close()


def test_np_symmetric_f32_near_recompute(H, orc):
    """Nothing stored but the partition: symmetric far field (one ACA per
    mirror pair, the mirror applied through V U^T), the near field evaluated
    in the product, FP32."""
    n, p0, eps = 20000, 0.05, 1e-5
    pts = synth.uniform_points(n, 3, 31, dtype=np.float32)
    x = synth.normal_vector(n, 32, dtype=np.float32)
    kw = dict(compute_dtype="f32", leaf_size=64, eta=1.5, aca_eps=eps, max_rank=48,
              symmetric_far=1, near_recompute=1)
    print("build: N=%d d=3 F32 symmetric far field, nothing stored" % n, flush=True)
    hs, hn = _pair(H, pts, "gaussian", p0, **kw)
    zs = hs.matvec(_dev(x)).double().cpu().numpy()
    zn = hn.matvec(_dev(x)).double().cpu().numpy()
    assert np.array_equal(hn.ranks(), hs.ranks())
    rows = synth.sample_rows(n, 512, 33)
    zd = orc.dense_matvec(pts, x, "gaussian", p0, rows=rows)
    e_s, e_d = _rel(zn, zs), _rel(zn[rows], zd)
    print("  NP vs stored %.2e, vs dense (512 rows) %.2e; handle %.1f MB vs %.1f MB"
          % (e_s, e_d, hn.stats().device_bytes / 1e6, hs.stats().device_bytes / 1e6), flush=True)
    assert e_s <= 2e-6
    assert e_d <= 10 * eps
    hs.close()
    hn.close()


def test_np_fixed_rank_alpha_beta_sigma2(H):
    """Fixed rank k (the paper's experiments), z = alpha (H + sigma2 I) x +
    beta z, against the stored handle."""
    n = 5000
    pts = synth.uniform_points(n, 2, 41)
    x = synth.normal_vector(n, 42)
    z0 = synth.normal_vector(n, 43)
    kw = dict(compute_dtype="f64", leaf_size=100, eta=1.5, aca_eps=0.0, max_rank=8,
              rank_mode="fixed", sigma2=0.25)
    hs, hn = _pair(H, pts, "matern32", 0.2, **kw)
    zs, zn = _dev(z0), _dev(z0)
    H.hmx_matvec(hs.h, _dev(x), zs, 0.5, -2.0)
    H.hmx_matvec(hn.h, _dev(x), zn, 0.5, -2.0)
    assert np.array_equal(hn.ranks(), hs.ranks())
    assert (hn.ranks() == 8).sum() > 0.9 * len(hn.ranks())
    e = _rel(zn.cpu().numpy(), zs.cpu().numpy())
    print("fixed rank 8, alpha 0.5, beta -2, sigma2 0.25: NP vs stored %.2e" % e, flush=True)
    assert e <= 1e-13
    hs.close()
    hn.close()


def test_np_many_workgroup_aca(H):
    """Blocks with clusters of 2048 or more points run their ACA on many
    workgroups (the split path); in the product without precomputation that
    path runs chunk by chunk too."""
    n, p0 = 32768, 0.02
    pts = synth.uniform_points(n, 2, 51)
    x = synth.normal_vector(n, 52)
    kw = dict(compute_dtype="f64", leaf_size=128, eta=1.5, aca_eps=1e-6, max_rank=32,
              aca_split_rows=2048)
    print("build: N=%d d=2 F64, split threshold 2048, stored and far_recompute" % n, flush=True)
    hs, hn = _pair(H, pts, "gaussian", p0, **kw)
    zs = hs.matvec(_dev(x)).cpu().numpy()
    zn = hn.matvec(_dev(x)).cpu().numpy()
    assert np.array_equal(hn.ranks(), hs.ranks())
    e = _rel(zn, zs)
    print("  NP vs stored %.2e" % e, flush=True)
    assert e <= 1e-13
    hs.close()
    hn.close()


def test_np_batched(H, orc):
    """Many problems in one block-diagonal handle without precomputation."""
    specs = [(1500, 2, 0.05), (3000, 3, 0.02), (2500, 2, 0.01)]
    pts = [synth.uniform_points(nq, d, 60 + q) for q, (nq, d, _) in enumerate(specs)]
    p0s = [p0 for (_, _, p0) in specs]
    kw = dict(compute_dtype="f64", leaf_size=64, eta=1.5, aca_eps=1e-7, max_rank=32)
    hs = H.HMatrix.batched([_dev(p) for p in pts], "gaussian", p0s, **kw)
    hn = H.HMatrix.batched([_dev(p) for p in pts], "gaussian", p0s, far_recompute=1, **kw)
    off = hs.offsets
    x = synth.normal_vector(int(off[-1]), 61)
    zs = hs.matvec(_dev(x)).cpu().numpy()
    zn = hn.matvec(_dev(x)).cpu().numpy()
    assert np.array_equal(hn.ranks(), hs.ranks())
    assert _rel(zn, zs) <= 1e-13
    for q, p in enumerate(pts):
        a, b = off[q], off[q + 1]
        assert _rel(zn[a:b], orc.dense_matvec(p, x[a:b], "gaussian", p0s[q])) <= 1e-6
    hs.close()
    hn.close()


def test_np_cg_and_unsupported(H):
    """CG on (H + sigma2 I) through the product without precomputation equals
    CG through the stored handle; graph capture, the allocation-free CG and
    the factor getter are refused."""
    n, p0, s2 = 3000, 0.05, 1.0
    pts = synth.uniform_points(n, 2, 71)
    b = _dev(synth.normal_vector(n, 72))
    kw = dict(compute_dtype="f64", leaf_size=64, eta=1.5, aca_eps=1e-8, max_rank=48, sigma2=s2,
              symmetric_far=1)
    hs, hn = _pair(H, pts, "gaussian", p0, **kw)
    xs, xn = torch.zeros_like(b), torch.zeros_like(b)
    rs = H.hmx_cg_solve(hs.h, b, xs, 1e-9, 2000)
    rn = H.hmx_cg_solve(hn.h, b, xn, 1e-9, 2000)
    print("CG stored: %s; CG far_recompute: %s" % (rs, rn), flush=True)
    e = _rel(xn.cpu().numpy(), xs.cpu().numpy())
    print("  solutions differ by %.2e" % e, flush=True)
    assert e <= 1e-8
    z = torch.empty_like(b)
    for call in (lambda: H.hmx_matvec_graph(hn.h, b, z),
                 lambda: H.hmx_cg_solve(hn.h, b, xn, 1e-6, 10, noalloc=True),
                 lambda: H.hmx_get_factors(hn.h, 0, n, n, 48)):
        with pytest.raises(H.HmxError) as ei:
            call()
        assert ei.value.status == H.HMX_ERR_UNSUPPORTED
    hs.close()
    hn.close()
