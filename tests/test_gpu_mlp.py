"""Rank predictor and learned rank sizing on the GPU, against the CPU oracle.

* The predictor's forward pass, its pinball-loss gradient (back-propagation
  in the library's own kernels) and Adam match the oracle's FP64 versions on
  the same FP32 weights and batch (relative 1e-4, FP32 arithmetic).
* The block features of a built H-matrix match the oracle's features of the
  same (bit-exact) partition.
* A learned build in the sizing form (prediction sizes storage, stopping test
  every step) equals the adaptive build bit for bit, whatever the prediction;
  in the one-shot form (target steps, test on the last term, adaptive
  continuation when it fails) it equals the oracle's one-shot ACA block by
  block, and its matvec keeps the plain method's error bound.
* A predictor trained on plain builds shrinks the ACA storage reserved up
  front several-fold and needs few fallbacks, at identical results.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NP = 8961


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
    return np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300)


def _features_data(n, seed):
    """Inputs shaped like block features (positive sizes, ratios, constants)."""
    g = synth.rng(seed)
    X = np.empty((n, 8))
    X[:, 0] = g.integers(5, 14, n)
    X[:, 1] = X[:, 0] + g.integers(-1, 2, n)
    X[:, 2] = synth.log_uniform(0.05, 20.0, n, seed + 1)
    X[:, 3] = X[:, 2] * (0.7 + 0.6 * g.random(n))
    X[:, 4] = synth.log_uniform(0.01, 50.0, n, seed + 2)
    X[:, 5] = np.minimum(X[:, 2], X[:, 3]) / X[:, 4]
    X[:, 6] = g.integers(2, 4, n)
    X[:, 7] = np.log10(synth.log_uniform(0.002, 0.05, n, seed + 3))
    y = g.integers(1, 40, n).astype(np.float64)
    return X.astype(np.float32), y.astype(np.float32)


def test_forward_matches_oracle(H, orc):
    w = synth.mlp_init_params(5)
    X, _ = _features_data(3000, 50)
    mlp = H.RankMLP(w)
    out = mlp.forward(_dev(X)).cpu().numpy()
    ref = orc.mlp_forward(w.astype(np.float64), X.astype(np.float64))
    err = _rel(out, ref)
    print("forward rel err %.3e" % err)
    assert err <= 1e-5
    # standardisation (x - mean) * scale applied on the device
    mean = X.mean(axis=0).astype(np.float32)
    scale = (1.0 / X.std(axis=0)).astype(np.float32)
    mlp.set_params(w, mean, scale)
    out = mlp.forward(_dev(X)).cpu().numpy()
    Xn = (X.astype(np.float64) - mean) * scale
    ref = orc.mlp_forward(w.astype(np.float64), Xn)
    assert _rel(out, ref) <= 1e-5
    w2, mu2, sc2 = mlp.get_params()
    assert np.array_equal(w2, w) and np.array_equal(mu2, mean) and np.array_equal(sc2, scale)
    mlp.close()


@pytest.mark.parametrize("B", [1, 37, 256, 1000, 4099])
def test_gradient_matches_oracle(H, orc, B):
    """Analytic back-propagation on the GPU vs the oracle's (pinned by
    central differences), same FP32 weights and batch."""
    w = synth.mlp_init_params(7)
    w[-1] = 3.0  # output bias near the targets: both signs of the residual occur
    X, y = _features_data(B, 60 + B)
    mean = X.mean(axis=0).astype(np.float32)
    sd = X.std(axis=0)
    scale = np.where(sd > 1e-6, 1.0 / np.maximum(sd, 1e-30), 1.0).astype(np.float32)
    mlp = H.RankMLP(w)
    mlp.set_params(w, mean, scale)
    loss, g = mlp.loss_grad(_dev(X), _dev(y), q=0.9)
    g = g.cpu().numpy().astype(np.float64)
    Xn = (X.astype(np.float64) - mean) * scale
    loss_o, g_o = orc.mlp_loss_grad(w.astype(np.float64), Xn, y.astype(np.float64), q=0.9)
    err = _rel(g, g_o)
    print("B=%d loss %.6g vs %.6g, grad rel err %.3e" % (B, loss, loss_o, err))
    assert abs(loss - loss_o) <= 1e-5 * abs(loss_o) + 1e-7
    assert err <= 1e-4
    mlp.close()


def test_adam_matches_oracle(H, orc):
    w = synth.mlp_init_params(9)
    mlp = H.RankMLP(w)
    wo = w.astype(np.float64)
    mo, vo = np.zeros(NP), np.zeros(NP)
    for t in range(1, 6):
        g = (synth.normal_vector(NP, 900 + t) * 10.0 ** (-t)).astype(np.float32)
        mlp.adam(_dev(g), lr=1e-2)
        orc.mlp_adam(wo, mo, vo, g.astype(np.float64), t, lr=1e-2)
    w_gpu = mlp.get_params()[0].astype(np.float64)
    err = np.abs(w_gpu - wo).max() / np.abs(wo).max()
    print("adam max rel dev %.3e" % err)
    assert err <= 1e-5
    mlp.close()


def test_train_loop_equals_steps(H, orc):
    """hmx_mlp_train = gather + loss_grad + adam per step, and follows the
    oracle's FP64 training on the same batches."""
    n, B, steps = 5000, 512, 20
    X, y = _features_data(n, 77)
    idx = synth.batch_indices(n, B, steps, 78)
    w = synth.mlp_init_params(11)
    mean = X.mean(axis=0).astype(np.float32)
    scale = (1.0 / X.std(axis=0)).astype(np.float32)
    a = H.RankMLP(w)
    a.set_params(w, mean, scale)
    losses = torch.zeros(steps, dtype=torch.float64, device="cuda:0")
    a.train(_dev(X), _dev(y), _dev(idx), B, steps, q=0.9, lr=3e-3, losses=losses)
    wa = a.get_params()[0]
    b = H.RankMLP(w)
    b.set_params(w, mean, scale)
    for s in range(steps):
        sl = idx[s * B:(s + 1) * B]
        _, g = b.loss_grad(_dev(X[sl]), _dev(y[sl]), q=0.9)
        b.adam(g, lr=3e-3)
    wb = b.get_params()[0]
    assert np.array_equal(wa, wb)
    # oracle training on the same batches (FP64)
    wo = w.astype(np.float64)
    mo, vo = np.zeros(NP), np.zeros(NP)
    Xn = (X.astype(np.float64) - mean) * scale
    lo = []
    for s in range(steps):
        sl = idx[s * B:(s + 1) * B]
        l, g = orc.mlp_loss_grad(wo, Xn[sl], y[sl].astype(np.float64), q=0.9)
        lo.append(l)
        orc.mlp_adam(wo, mo, vo, g, s + 1, lr=3e-3)
    lg = losses.cpu().numpy()
    print("losses gpu", lg[:3], lg[-3:], "oracle", lo[:3], lo[-3:])
    assert np.allclose(lg, lo, rtol=1e-3, atol=1e-5)
    assert _rel(wa, wo) <= 1e-3
    assert lg[-1] < lg[0]
    a.close()
    b.close()


def test_checkpoint_resumes_training_bit_for_bit(H, tmp_path):
    """hmx_mlp_save / hmx_mlp_load: a predictor saved after 10 training steps
    and loaded again holds the same parameters and standardisation, predicts
    the same, and its next 10 steps (Adam moments and step count restored)
    equal 20 uninterrupted steps bit for bit."""
    n, B = 4000, 256
    X, y = _features_data(n, 81)
    idx = synth.batch_indices(n, B, 20, 82)
    w = synth.mlp_init_params(13)
    mean = X.mean(axis=0).astype(np.float32)
    scale = (1.0 / X.std(axis=0)).astype(np.float32)
    Xd, yd, idd = _dev(X), _dev(y), _dev(idx)
    a = H.RankMLP(w)
    a.set_params(w, mean, scale)
    a.train(Xd, yd, idd, B, 20, q=0.9, lr=3e-3)
    b = H.RankMLP(w)
    b.set_params(w, mean, scale)
    b.train(Xd, yd, idd[:10 * B].contiguous(), B, 10, q=0.9, lr=3e-3)
    path = tmp_path / "predictor.bin"
    b.save(path)
    assert path.stat().st_size == 8 + 16 + 4 * (3 * NP + 16)
    c = H.RankMLP.load(path)
    for u, v in zip(b.get_params(), c.get_params()):
        assert np.array_equal(u, v)
    assert torch.equal(b.forward(Xd), c.forward(Xd))
    c.train(Xd, yd, idd[10 * B:].contiguous(), B, 10, q=0.9, lr=3e-3)
    assert np.array_equal(a.get_params()[0], c.get_params()[0])
    for m in (a, b, c):
        m.close()


def test_invalid_arguments(H):
    mlp = H.RankMLP()
    X = torch.zeros((4, 8), dtype=torch.float32, device="cuda:0")
    y = torch.zeros(4, dtype=torch.float32, device="cuda:0")
    with pytest.raises(H.HmxError):
        mlp.loss_grad(X, y, q=1.5)
    with pytest.raises(H.HmxError):
        H.hmx_build(_dev(synth.uniform_points(100, 2, 1)), H.make_kernel("gaussian", 0.1),
                    H.hmx_params_default(rank_mode="learned"))
    mlp.close()


def _oracle_features(orc, pts, adm, ell):
    _, _, soa = orc.order(pts)
    F = np.empty((len(adm), 8))
    for q, b in enumerate(adm):
        ta, tb = soa[:, b[0]:b[1]].min(axis=1), soa[:, b[0]:b[1]].max(axis=1)
        sa, sb = soa[:, b[2]:b[3]].min(axis=1), soa[:, b[2]:b[3]].max(axis=1)
        F[q] = orc.features(ta, tb, sa, sb, b[1] - b[0], b[3] - b[2], ell)
    return F


@pytest.mark.parametrize("d,kernel,p0", [(2, "gaussian", 0.01), (3, "matern32", 0.2)])
def test_block_features_match_oracle(H, orc, d, kernel, p0):
    pts = synth.uniform_points(6000, d, 300 + d)
    hm = H.HMatrix(_dev(pts), kernel, p0, compute_dtype="f32", leaf_size=64, eta=1.5,
                   aca_eps=1e-5, max_rank=32)
    F, yr = H.hmx_block_features(hm.h)
    F = F.cpu().numpy()
    part = hm.partition()
    ell = np.sqrt(p0) if kernel == "gaussian" else p0
    Fo = _oracle_features(orc, pts, part["adm"], ell).astype(np.float32)
    dev = np.abs(F - Fo) / np.maximum(np.abs(Fo), 1e-30)
    print("features: %d blocks, max rel dev %.3e" % (len(F), dev.max()))
    assert dev.max() <= 2.0 ** -23
    assert np.array_equal(yr.cpu().numpy(), hm.ranks().astype(np.float32))
    hm.close()


def _const_predictor(H, c):
    w = np.zeros(NP, np.float32)
    w[-1] = c  # output bias only: prediction c for every block
    return H.RankMLP(w)


@pytest.mark.parametrize("c", [0.5, 6.0, 200.0])
def test_learned_sizing_equals_adaptive(H, orc, c):
    """Sizing form: whatever the prediction, ranks and matvec are those of
    the adaptive method (too small a target only costs a second pass)."""
    n, eps, kmax = 4096, 1e-6, 32
    pts = synth.uniform_points(n, 2, 11)
    x = _dev(synth.normal_vector(n, 12))
    mlp = _const_predictor(H, c)
    kw = dict(compute_dtype="f64", leaf_size=64, eta=1.5, aca_eps=eps, max_rank=kmax)
    ha = H.HMatrix(_dev(pts), "gaussian", 0.1, **kw)
    hl = H.HMatrix(_dev(pts), "gaussian", 0.1, rank_mode="learned", mlp=mlp, aca_chunk_mb=1, **kw)
    sa, sl = ha.stats(), hl.stats()
    print("c=%g: fallbacks %d of %d, capacity %d vs %d, chunks %d vs %d"
          % (c, sl.aca_fallback, sl.n_adm, sl.aca_capacity, sa.aca_capacity, sl.aca_chunks,
             sa.aca_chunks))
    assert np.array_equal(ha.ranks(), hl.ranks())
    assert torch.equal(ha.matvec(x), hl.matvec(x))
    if c > 100:
        assert sl.aca_fallback == 0
    ha.close()
    hl.close()
    mlp.close()


@pytest.mark.parametrize("c", [0.5, 4.0, 200.0])
def test_learned_one_shot_equals_oracle(H, orc, c):
    """A constant predictor c gives target r^ = clamp(ceil(c) + 1, 1, R):
    every block must equal the oracle's one-shot ACA with that target."""
    n, eps, kmax = 4096, 1e-6, 32
    pts = synth.uniform_points(n, 2, 11)
    x = synth.normal_vector(n, 12)
    mlp = _const_predictor(H, c)
    hm = H.HMatrix(_dev(pts), "gaussian", 0.1, compute_dtype="f64", leaf_size=64, eta=1.5,
                   aca_eps=eps, max_rank=kmax, rank_mode="learned", mlp=mlp,
                   learned_one_shot=1, aca_chunk_mb=1)
    s = hm.stats()
    ranks = hm.ranks()
    part = hm.partition()
    _, _, soa = orc.order(pts)
    target = int(np.ceil(c)) + 1
    ro = np.empty(len(ranks), np.int32)
    fallback = 0
    for q, b in enumerate(part["adm"]):
        R = min(kmax, b[1] - b[0], b[3] - b[2])
        t = min(target, R)
        _, _, r, _ = orc.aca(soa, "gaussian", 0.1, *b[:4], kmax, eps, r_start=t)
        ro[q] = r
        fallback += r > t
    agree = np.mean(ranks == ro)
    print("c=%g target %d: rank agreement %.4f, overflows %d + fallbacks %d (oracle > target: "
          "%d), chunks %d" % (c, target, agree, s.aca_overflow, s.aca_fallback, fallback,
                              s.aca_chunks))
    assert agree >= 0.97 and np.abs(ranks.astype(int) - ro).max() <= 2
    # every block that went past its target either continued in overflow
    # storage or was approximated again
    assert s.aca_overflow + s.aca_fallback >= fallback
    z = hm.matvec(_dev(x)).cpu().numpy()
    zd = orc.dense_matvec(pts, x, "gaussian", 0.1)
    err = _rel(z, zd)
    print("matvec rel err %.3e" % err)
    assert err <= 10 * eps + 4 * 2.0 ** -53
    hm.close()
    mlp.close()


def _train_predictor(H, builds, d, seed, steps=600, batch=1024, q=0.9):
    """Train on (features, rank) pairs of plain ACA-only builds."""
    Xs, ys = [], []
    for k, (n, p0) in enumerate(builds):
        pts = synth.uniform_points(n, d, seed + k)
        hm = H.HMatrix(_dev(pts), "gaussian", p0, compute_dtype="f32", leaf_size=64, eta=1.5,
                       aca_eps=1e-5, max_rank=64, aca_only=1)
        F, y = H.hmx_block_features(hm.h)
        Xs.append(F.clone())
        ys.append(y.clone())
        hm.close()
    X = torch.cat(Xs)
    y = torch.cat(ys)
    mlp = H.RankMLP(synth.mlp_init_params(seed))
    mlp.fit_normalization(X)
    idx = _dev(synth.batch_indices(X.shape[0], batch, steps, seed + 99))
    losses = torch.zeros(steps, dtype=torch.float64, device="cuda:0")
    mlp.train(X, y, idx, batch, steps, q=q, lr=3e-3, losses=losses)
    lh = losses.cpu().numpy()
    print("trained on %d pairs: loss %.3f -> %.3f" % (X.shape[0], lh[:20].mean(), lh[-20:].mean()))
    assert lh[-20:].mean() < 0.5 * lh[:20].mean()
    return mlp


def test_trained_predictor_gain(H, orc):
    """What the trained predictor gains over the method without it: ACA
    storage reserved up front (capacity) shrinks several-fold against k_max
    sizing and few blocks fall back, with results identical to the adaptive
    method (whose matvec error is within the tolerance)."""
    d = 3
    p0s = synth.log_uniform(0.002, 0.05, 12, 7001)
    ns = np.round(2.0 ** (12 + 3 * synth.rng(7002).random(12))).astype(int)
    mlp = _train_predictor(H, list(zip(ns, p0s)), d, 7100)
    n, p0 = 30000, 0.01
    pts = synth.uniform_points(n, d, 7200, dtype=np.float32)
    x = synth.normal_vector(n, 7201, dtype=np.float32)
    rows = synth.sample_rows(n, 256, 7202)
    zd = orc.dense_matvec(pts, x, "gaussian", p0, rows=rows)
    res = {}
    for mode in ("adaptive", "learned"):
        kw = dict(mlp=mlp) if mode == "learned" else {}
        hm = H.HMatrix(_dev(pts), "gaussian", p0, compute_dtype="f32", leaf_size=64, eta=1.5,
                       aca_eps=1e-5, max_rank=64, rank_mode=mode, **kw)
        s = hm.stats()
        zf = hm.matvec(_dev(x)).double().cpu().numpy()
        z = zf[rows]
        res[mode] = dict(err=_rel(z, zd), cap=s.aca_capacity, fb=s.aca_fallback, n_adm=s.n_adm,
                         chunks=s.aca_chunks, sum_rank=s.sum_rank, aca_ms=s.phase_ms[3],
                         ranks=hm.ranks(), z=zf)
        hm.close()
    a, l = res["adaptive"], res["learned"]
    print({k: {q: v for q, v in r.items() if q not in ("ranks", "z")} for k, r in res.items()})
    assert np.array_equal(a["ranks"], l["ranks"]) and np.array_equal(a["z"], l["z"])
    assert a["err"] <= 1e-4
    assert l["cap"] <= 0.6 * a["cap"]
    assert l["fb"] <= 0.15 * l["n_adm"]
    mlp.close()


@pytest.mark.parametrize("d,kernel,p0", [(2, "gaussian", 0.01), (3, "matern32", 0.15)])
def test_fused_inference_matches_oracle(H, orc, d, kernel, p0):
    """The hand-written in-build inference (features, standardisation, four
    layers, target clamp in one kernel) against the oracle's FP64 forward on
    the oracle's features of the same partition, with He-initialised weights,
    random biases and a non-trivial standardisation: a transposed weight
    index, a wrong bias or standardisation fails the comparison."""
    n, kmax = 30000, 48
    pts = synth.uniform_points(n, d, 8100 + d, dtype=np.float32)
    hm = H.HMatrix(_dev(pts), kernel, p0, compute_dtype="f32", leaf_size=64, eta=1.5,
                   aca_eps=1e-4, max_rank=kmax, aca_only=1)
    w = synth.mlp_init_params(8200 + d).astype(np.float64)
    g = synth.rng(8300 + d)
    # random biases (the He initialisation leaves them zero)
    offs = np.cumsum([0] + [a * b + b for a, b in zip((8, 64, 64, 64), (64, 64, 64, 1))])
    for lay, (fi, fo) in enumerate(zip((8, 64, 64, 64), (64, 64, 64, 1))):
        w[offs[lay] + fi * fo: offs[lay + 1]] = 0.3 * g.standard_normal(fo)
    w[-65:-1] *= 3.0  # output layer: spread the outputs over several integer targets
    w[-1] = 6.0  # centre the outputs where the target clamp is active
    w = w.astype(np.float32)
    part = hm.partition()
    ell = np.sqrt(p0) if kernel == "gaussian" else p0
    Fo = _oracle_features(orc, pts.astype(np.float64), part["adm"], ell).astype(np.float32)
    mean = (Fo.mean(axis=0) + 0.1 * g.standard_normal(8)).astype(np.float32)
    scale = (1.0 / (Fo.std(axis=0) + 0.5) * (0.8 + 0.4 * g.random(8))).astype(np.float32)
    mlp = H.RankMLP(w)
    mlp.set_params(w, mean, scale)
    pred, tgt = H.hmx_rank_predict(hm.h, mlp)
    pred, tgt = pred.cpu().numpy().astype(np.float64), tgt.cpu().numpy()
    Xs = (Fo.astype(np.float64) - mean) * scale
    o = orc.mlp_forward(w, Xs)
    dev = np.abs(pred - o) / (1.0 + np.abs(o))
    print("fused inference: %d blocks, outputs in [%.2f, %.2f], max dev %.3e"
          % (len(o), o.min(), o.max(), dev.max()))
    assert len(o) > 1000 and o.std() > 1.0
    assert dev.max() <= 1e-5
    adm = part["adm"]
    R = np.minimum(np.minimum(adm[:, 1] - adm[:, 0], adm[:, 3] - adm[:, 2]), kmax)
    want = np.clip(np.ceil(o) + 1, 1, R).astype(np.int32)
    near_int = np.abs(o - np.round(o)) <= 1e-5 * (1.0 + np.abs(o))
    print("targets: %d of %d differ, %d outputs within 1e-5 of an integer"
          % (np.sum(tgt != want), len(o), near_int.sum()))
    assert np.array_equal(tgt[~near_int], want[~near_int])
    assert np.all(np.abs(tgt[near_int] - want[near_int]) <= 1)
    assert np.all((tgt >= 1) & (tgt <= R))
    hm.close()
    mlp.close()
