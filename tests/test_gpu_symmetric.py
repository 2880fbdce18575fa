"""The symmetric far field on the GPU against the oracle's symmetric mode.

With symmetric_far = 1 only the admissible leaf with tau before sigma is
approximated; its mirror (sigma, tau) uses the transposed factors, and phase
1 of the matvec reads every V from the mirror's row-tile factor pieces.
Checked here: the partition is unchanged, ranks against the oracle (every
difference a near tie of Algorithm 2's decisions), mirrors carry their
primary's factors transposed bit for bit, the stored factor entries are
those of the primary leaves only, the operator is symmetric to rounding, the
product meets the tolerance against the dense product and the oracle's
symmetric product, in FP64, FP32 and BF16, and with learned sizing, the
no-storage near field, many problems in one handle and CG.
"""
import numpy as np
import pytest

import aca_ties
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


def test_symmetric_f64_against_oracle(H, orc):
    n, p0, leaf, eta, eps, kmax = 4096, 0.1, 64, 1.5, 1e-6, 32
    pts = synth.uniform_points(n, 2, 11)
    x = synth.normal_vector(n, 12)
    y = synth.normal_vector(n, 13)
    print("build: N=%d FP64 symmetric far field" % n, flush=True)
    hs = H.HMatrix(_dev(pts), "gaussian", p0, compute_dtype="f64", leaf_size=leaf, eta=eta,
                   aca_eps=eps, max_rank=kmax, symmetric_far=1)
    hp = H.HMatrix(_dev(pts), "gaussian", p0, compute_dtype="f64", leaf_size=leaf, eta=eta,
                   aca_eps=eps, max_rank=kmax)
    ps, pp = hs.partition(), hp.partition()
    assert np.array_equal(ps["adm"], pp["adm"]) and np.array_equal(ps["dense"], pp["dense"])
    adm = ps["adm"]
    ranks = hs.ranks()
    zo, ro, sto = orc.hmvp(pts, x, "gaussian", p0, leaf, eta, kmax, eps, symmetric=True,
                           want_ranks=True)
    # ranks: mirrors equal their primaries; primaries the oracle's up to near ties
    key = {(int(b[0]), int(b[2])): q for q, b in enumerate(adm)}
    mirror = np.array([key[(int(b[2]), int(b[0]))] for b in adm])
    assert np.array_equal(ranks, ranks[mirror])
    prim = adm[:, 0] <= adm[:, 2]
    _, _, soa = orc.order(pts)
    bad = np.where(prim & (ranks != ro))[0]
    print("primary ranks differing from the oracle: %d of %d" % (len(bad), prim.sum()))
    for q in bad:
        b = adm[q]
        m, nn = b[1] - b[0], b[3] - b[2]
        Ug, Vg, rg = H.hmx_get_factors(hs.h, int(q), m, nn, kmax)
        Uo, Vo, r_o, _, tr = orc.aca(soa, "gaussian", p0, *b[:4], kmax, eps, eps0=1e-14,
                                     want_trace=True)
        s = aca_ties.first_divergence(Ug, Vg, Uo, Vo)
        what, gap = aca_ties.explain(tr, s, rg, r_o, 1e-6)
        print("  block %d: GPU %d oracle %d, step %d %s gap %.2e" % (q, rg, r_o, s, what, gap))
        assert gap <= 1e-6
    # a mirror's factors are its primary's, transposed, bit for bit
    for q in np.where(prim)[0][:: max(1, prim.sum() // 12)]:
        b = adm[q]
        m, nn = b[1] - b[0], b[3] - b[2]
        U, V, r = H.hmx_get_factors(hs.h, int(q), m, nn, kmax)
        Um, Vm, rm = H.hmx_get_factors(hs.h, int(mirror[q]), nn, m, kmax)
        assert r == rm and np.array_equal(Um, V) and np.array_equal(Vm, U)
    # storage: the primary leaves' factors only; both phases read them all
    st = hs.stats()
    r64 = ranks.astype(np.int64)
    m_, n_ = (adm[:, 1] - adm[:, 0]).astype(np.int64), (adm[:, 3] - adm[:, 2]).astype(np.int64)
    assert st.factor_entries == int(np.sum((r64 * (m_ + n_))[prim]))
    assert st.u_entries == int(np.sum(r64 * m_)) and st.v_entries == int(np.sum(r64 * n_))
    assert st.factor_entries < 0.55 * hp.stats().factor_entries
    # the product: oracle's symmetric product, dense product, symmetry
    zx = hs.matvec(_dev(x)).cpu().numpy()
    zy = hs.matvec(_dev(y)).cpu().numpy()
    zd = orc.dense_matvec(pts, x, "gaussian", p0)
    e_o, e_d = _rel(zx, zo), _rel(zx, zd)
    asym = abs(y @ zx - x @ zy) / (np.linalg.norm(y) * np.linalg.norm(zx))
    zxp = hp.matvec(_dev(x)).cpu().numpy()
    zyp = hp.matvec(_dev(y)).cpu().numpy()
    asym_p = abs(y @ zxp - x @ zyp) / (np.linalg.norm(y) * np.linalg.norm(zxp))
    print("symmetric FP64: vs oracle %.2e, vs dense %.2e, asymmetry %.2e (two-sided %.2e)"
          % (e_o, e_d, asym, asym_p))
    assert e_o <= 10 * eps and e_d <= 10 * eps
    assert asym <= 1e-14 and asym_p > 100 * asym
    hs.close()
    hp.close()


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_symmetric_f32_bf16(H, orc, storage):
    n, p0, eps = 30000, 0.02, 1e-5
    pts = synth.uniform_points(n, 3, 4501, dtype=np.float32)
    x = synth.normal_vector(n, 4502, dtype=np.float32)
    y = synth.normal_vector(n, 4503, dtype=np.float32)
    print("build: N=%d 3-d %s symmetric far field" % (n, storage), flush=True)
    hs = H.HMatrix(_dev(pts), "gaussian", p0, compute_dtype="f32", storage_dtype=storage,
                   leaf_size=64, eta=1.5, aca_eps=eps, max_rank=64, symmetric_far=1)
    rows = synth.sample_rows(n, 512, 4504)
    zd = orc.dense_matvec(pts, x, "gaussian", p0, rows=rows)
    zx = hs.matvec(_dev(x)).double().cpu().numpy()
    zy = hs.matvec(_dev(y)).double().cpu().numpy()
    err = _rel(zx[rows], zd)
    asym = abs(y.astype(np.float64) @ zx - x.astype(np.float64) @ zy) / (
        np.linalg.norm(y) * np.linalg.norm(zx))
    u = 2.0 ** -24 if storage == "f32" else 2.0 ** -9
    print("symmetric %s: sampled-row err %.3e, asymmetry %.2e" % (storage, err, asym))
    assert err <= 10 * eps + 4 * u
    assert asym <= 1e-5
    hs.close()


def test_symmetric_learned_recompute_batched(H):
    """Learned sizing keeps the symmetric build's ranks and product bits; the
    no-storage near field gives the stored product within FP32 rounding (the
    entries are evaluated by another instance of the same formula, whose
    compiled FP32 exponent argument can differ in the last bit); two problems
    in one handle give each problem's product."""
    n, p0 = 20000, 0.01
    pts = synth.uniform_points(n, 2, 4601, dtype=np.float32)
    x = _dev(synth.normal_vector(n, 4602, dtype=np.float32))
    kw = dict(compute_dtype="f32", leaf_size=64, eta=1.5, aca_eps=1e-5, max_rank=48,
              symmetric_far=1)
    w = np.zeros(8961, np.float32)
    w[-1] = 3.0
    mlp = H.RankMLP(w)
    ha = H.HMatrix(_dev(pts), "gaussian", p0, **kw)
    hl = H.HMatrix(_dev(pts), "gaussian", p0, rank_mode="learned", mlp=mlp, aca_chunk_mb=1, **kw)
    hr = H.HMatrix(_dev(pts), "gaussian", p0, near_recompute=1, **kw)
    za = ha.matvec(x)
    assert np.array_equal(ha.ranks(), hl.ranks()) and torch.equal(za, hl.matvec(x))
    zr = hr.matvec(x)
    dev = (torch.linalg.norm((zr - za).double()) / torch.linalg.norm(za.double())).item()
    print("no-storage near field vs stored: %.2e" % dev)
    assert dev <= 1e-6
    pts2 = synth.uniform_points(n // 2, 3, 4603, dtype=np.float32)
    h2 = H.HMatrix(_dev(pts2), "gaussian", p0, **kw)
    x2 = _dev(synth.normal_vector(n // 2, 4604, dtype=np.float32))
    hb = H.HMatrix.batched([_dev(pts), _dev(pts2)], "gaussian", [p0, p0], **kw)
    zb = hb.matvec(torch.cat([x, x2]))
    for zq, zs in ((zb[:n], za), (zb[n:], h2.matvec(x2))):
        dev = (torch.linalg.norm((zq - zs).double()) / torch.linalg.norm(zs.double())).item()
        print("batched vs single: %.2e" % dev)
        assert dev <= 1e-5
    for h in (ha, hl, hr, h2, hb):
        h.close()
    mlp.close()


def test_symmetric_coincident_points(H):
    """Clusters of coincident points are their own mirror (tau = sigma, zero
    diameter, admissible): such a leaf keeps its own V."""
    pts = np.full((1000, 2), 0.25)
    hm = H.HMatrix(_dev(pts), "lowrank", 1.0, compute_dtype="f64", leaf_size=16, eta=1.5,
                   aca_eps=1e-8, symmetric_far=1)
    assert hm.partition()["adm"].tolist() == [[0, 1000, 0, 1000, 0]]
    x = synth.normal_vector(1000, 3)
    z = hm.matvec(_dev(x)).cpu().numpy()
    c = (1.0 + 2 * 0.25 ** 2) ** 2  # (1 + y.y)^2 for every pair
    assert np.allclose(z, c * x.sum(), rtol=1e-12, atol=1e-10)
    hm.close()


def test_symmetric_cg_krr(H, orc):
    """CG on the symmetric operator (H + sigma2 I) c = y (kernel ridge
    regression, Matern-3/2 l = 0.1, sigma2 = 1e-2, GMM points in [0,1]^3)
    against the oracle's dense CG."""
    n = 3000
    pts = synth.gmm_points(n, 3, 31, ncomp=16)
    y = synth.krr_target(pts, 32)
    hm = H.HMatrix(_dev(pts), "matern32", 0.1, compute_dtype="f64", leaf_size=64, eta=1.5,
                   aca_eps=1e-9, max_rank=96, sigma2=1e-2, symmetric_far=1)
    c = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    s, it, res, tres = H.hmx_cg_solve(hm.h, _dev(y), c, rel_tol=1e-9, max_iter=2000)
    print("cg symmetric f64: iters %d rel res %.3e true %.3e" % (it, res, tres))
    assert s == H.HMX_OK and res <= 1e-9 and tres <= 1e-7
    c_ref, rc, _, _ = orc.cg_dense(pts, y, "matern32", 0.1, 1e-2, tol=1e-12)
    err = np.linalg.norm(c.cpu().numpy() - c_ref) / np.linalg.norm(c_ref)
    print("vs dense CG: %.3e" % err)
    assert err <= 1e-4
    hm.close()
