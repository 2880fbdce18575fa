"""Batched build of many independent problems as one block-diagonal handle.

Each problem's ordering and block partition, read out of the union, must
equal the oracle's for that problem bit for bit; each problem's slice of the
union matvec must match its own FP64 dense product within the tolerance; a
learned (sizing-form) batch must equal the adaptive batch bit for bit.
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
    return np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b)


def _problems(specs, seed, dtype=np.float64):
    pts = [synth.uniform_points(n, d, seed + q, dtype=dtype) for q, (n, d, _) in enumerate(specs)]
    return pts, [p0 for (_, _, p0) in specs]


SPECS = [(1000, 2, 0.05), (3000, 3, 0.02), (5000, 2, 0.01), (777, 3, 0.1), (2048, 1, 0.03),
         (4096, 2, 0.005)]


def test_batched_partition_and_matvec_f64(H, orc):
    pts, p0s = _problems(SPECS, 500)
    leaf, eta, eps, kmax = 64, 1.5, 1e-7, 48
    hm = H.HMatrix.batched([_dev(p) for p in pts], "gaussian", p0s, compute_dtype="f64",
                           leaf_size=leaf, eta=eta, aca_eps=eps, max_rank=kmax)
    off = hm.offsets
    assert list(off) == list(np.cumsum([0] + [s[0] for s in SPECS]))
    part = hm.partition()
    x = synth.normal_vector(int(off[-1]), 501)
    z = hm.matvec(_dev(x)).cpu().numpy()
    for q, p in enumerate(pts):
        a, b = off[q], off[q + 1]
        codes, perm, soa = orc.order(p)
        assert np.array_equal(part["codes"][a:b], codes)
        assert np.array_equal(part["perm"][a:b] - a, perm)
        adm_o, den_o, _ = orc.partition(soa, leaf, eta)
        sel = (part["adm"][:, 0] >= a) & (part["adm"][:, 0] < b)
        adm = part["adm"][sel].copy()
        adm[:, :4] -= a
        assert np.array_equal(adm, adm_o), q
        sel = (part["dense"][:, 0] >= a) & (part["dense"][:, 0] < b)
        den = part["dense"][sel].copy()
        den[:, :4] -= a
        assert np.array_equal(den, den_o), q
        zd = orc.dense_matvec(p, x[a:b], "gaussian", p0s[q])
        err = _rel(z[a:b], zd)
        print("problem %d: n %d d %d p0 %g  adm %d dense %d  rel err %.3e"
              % (q, b - a, p.shape[1], p0s[q], len(adm_o), len(den_o), err))
        assert err <= 10 * eps + 1e-12
    hm.close()


def test_batched_f32_like_uneven_workload(H, orc):
    """Uneven sizes, d in {2, 3}, p0 log-uniform: every problem's slice
    against its own dense product, and against an individual build."""
    g = synth.rng(4100)
    nprob = 16
    ns = np.round(2.0 ** (10 + 3 * g.random(nprob))).astype(int)
    ds = g.integers(2, 4, nprob)
    p0s = synth.log_uniform(0.005, 0.05, nprob, 4101)
    pts = [synth.uniform_points(int(ns[q]), int(ds[q]), 4200 + q, dtype=np.float32)
           for q in range(nprob)]
    kw = dict(compute_dtype="f32", leaf_size=128, eta=1.5, aca_eps=1e-5, max_rank=64)
    hm = H.HMatrix.batched([_dev(p) for p in pts], "gaussian", list(p0s), **kw)
    off = hm.offsets
    x = synth.normal_vector(int(off[-1]), 4300, dtype=np.float32)
    z = hm.matvec(_dev(x)).double().cpu().numpy()
    s = hm.stats()
    print("batch: %d points, %d adm, %d dense, %d tiles, aca %.1f ms"
          % (off[-1], s.n_adm, s.n_dense, s.n_tiles, s.phase_ms[3]))
    for q in range(nprob):
        a, b = off[q], off[q + 1]
        zd = orc.dense_matvec(pts[q], x[a:b], "gaussian", p0s[q])
        err = _rel(z[a:b], zd)
        one = H.HMatrix(_dev(pts[q]), "gaussian", float(p0s[q]), **kw)
        zi = one.matvec(_dev(x[a:b])).double().cpu().numpy()
        erri = _rel(zi, zd)
        one.close()
        print("problem %2d: n %5d d %d p0 %.4f  batched err %.3e  single err %.3e"
              % (q, b - a, ds[q], p0s[q], err, erri))
        # below 1e-6 both errors are FP32 rounding of the row sums, whose
        # order depends on the row-tile grid (the batched handle and the
        # single ones may use different default grids)
        assert err <= 1e-4 and err <= 3 * max(erri, 1e-6)
    hm.close()


def test_batched_learned_equals_adaptive(H):
    pts, p0s = _problems(SPECS, 600, np.float32)
    w = np.zeros(8961, np.float32)
    w[-1] = 3.0
    mlp = H.RankMLP(w)
    kw = dict(compute_dtype="f32", leaf_size=64, eta=1.5, aca_eps=1e-5, max_rank=32)
    ha = H.HMatrix.batched([_dev(p) for p in pts], "gaussian", p0s, **kw)
    hl = H.HMatrix.batched([_dev(p) for p in pts], "gaussian", p0s, rank_mode="learned", mlp=mlp,
                           **kw)
    x = _dev(synth.normal_vector(int(ha.offsets[-1]), 601, dtype=np.float32))
    assert np.array_equal(ha.ranks(), hl.ranks())
    assert torch.equal(ha.matvec(x), hl.matvec(x))
    print("fallbacks %d of %d" % (hl.stats().aca_fallback, hl.stats().n_adm))
    ha.close()
    hl.close()
    mlp.close()


def test_batched_invalid(H):
    a = _dev(synth.uniform_points(100, 2, 1))
    b = _dev(synth.uniform_points(100, 2, 2))
    p = H.hmx_params_default()
    with pytest.raises(H.HmxError) as e:
        H.hmx_build_batched([a, b], [H.make_kernel("gaussian", 0.1), H.make_kernel("matern32", 0.1)],
                            p)
    assert e.value.status == H.HMX_ERR_INVALID_ARG
    with pytest.raises(H.HmxError) as e:
        H.hmx_build_batched([a, b], [H.make_kernel("lowrank"), H.make_kernel("lowrank")], p)
    assert e.value.status == H.HMX_ERR_UNSUPPORTED
    h, off = H.hmx_build_batched([a], [H.make_kernel("gaussian", 0.1)], p)
    assert list(off) == [0, 100]
    with pytest.raises(H.HmxError):
        H.hmx_block_features(h)
    H.hmx_destroy(h)


def test_matvec_batched_over_separate_handles(H):
    """hmx_matvec_batched over separately built handles equals one
    hmx_matvec per handle, bit for bit, with alpha and beta."""
    specs = [(3000, 2, 0.02), (5000, 3, 0.05), (1200, 2, 0.01)]
    hs, xs, zs, zr = [], [], [], []
    for q, (n, d, p0) in enumerate(specs):
        pts = synth.uniform_points(n, d, 700 + q, dtype=np.float32)
        hs.append(H.HMatrix(_dev(pts), "gaussian", p0, compute_dtype="f32", leaf_size=64,
                            eta=1.5, aca_eps=1e-5, max_rank=32))
        xs.append(_dev(synth.normal_vector(n, 710 + q, dtype=np.float32)))
        z0 = _dev(synth.normal_vector(n, 720 + q, dtype=np.float32))
        zs.append(z0.clone())
        zr.append(z0.clone())
    H.hmx_matvec_batched([h.h for h in hs], xs, zs, alpha=0.5, beta=-2.0)
    for h, x, z in zip(hs, xs, zr):
        H.hmx_matvec(h.h, x, z, 0.5, -2.0)
    for a, b in zip(zs, zr):
        assert torch.equal(a, b)
    with pytest.raises(ValueError):
        H.hmx_matvec_batched([h.h for h in hs], xs[:2], zs[:2] + [xs[0]])
    for h in hs:
        h.close()
