"""Near field recomputed in every product (no storage) against the stored
near field and the FP64 dense product."""
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
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


@pytest.mark.parametrize("dtype,storage,kernel,d,n,leaf", [
    ("f64", "f64", "gaussian", 2, 4096, 64),
    ("f32", "f32", "gaussian", 3, 20000, 100),
    ("f32", "bf16", "matern32", 2, 15000, 64),
    ("f32", "f32", "gaussian", 1, 3001, 16),
])
def test_recompute_matches_stored(H, orc, dtype, storage, kernel, d, n, leaf):
    npdt = np.float64 if dtype == "f64" else np.float32
    pts = synth.uniform_points(n, d, 700 + d, dtype=npdt)
    x = synth.normal_vector(n, 701, dtype=npdt)
    p0 = 0.05 if kernel == "gaussian" else 0.2
    kw = dict(compute_dtype=dtype, storage_dtype=storage, leaf_size=leaf, eta=1.5,
              aca_eps=1e-6 if dtype == "f64" else 1e-5, max_rank=48, sigma2=0.1)
    hs = H.HMatrix(_dev(pts), kernel, p0, **kw)
    hr = H.HMatrix(_dev(pts), kernel, p0, near_recompute=1, **kw)
    ss, sr = hs.stats(), hr.stats()
    assert sr.near_entry_bytes == 0 and sr.near_entries == ss.near_entries
    assert sr.device_bytes < ss.device_bytes
    zs = hs.matvec(_dev(x)).double().cpu().numpy()
    zr = hr.matvec(_dev(x)).double().cpu().numpy()
    dev = _rel(zr, zs)
    rows = synth.sample_rows(n, 300, 702)
    zd = orc.dense_matvec(pts, x, kernel, p0, sigma2=0.1, rows=rows)
    err = _rel(zr[rows], zd)
    print("%s/%s %s d=%d: recompute vs stored %.3e, vs dense %.3e, device bytes %d vs %d"
          % (dtype, storage, kernel, d, dev, err, sr.device_bytes, ss.device_bytes))
    assert dev <= (1e-13 if dtype == "f64" else (3e-3 if storage == "bf16" else 1e-6))
    assert err <= (1e-5 if dtype == "f64" else (1e-2 if storage == "bf16" else 1e-4))
    hs.close()
    hr.close()


def test_recompute_batched_and_tiles(H, orc):
    specs = [(3000, 2, 0.02), (5000, 3, 0.01), (1500, 2, 0.05)]
    pts = [synth.uniform_points(nn, dd, 710 + q, dtype=np.float32)
           for q, (nn, dd, _) in enumerate(specs)]
    p0s = [p for (_, _, p) in specs]
    kw = dict(compute_dtype="f32", leaf_size=64, eta=1.5, aca_eps=1e-5, max_rank=32)
    hs = H.HMatrix.batched([_dev(p) for p in pts], "gaussian", p0s, **kw)
    hr = H.HMatrix.batched([_dev(p) for p in pts], "gaussian", p0s, near_recompute=1, **kw)
    off = hs.offsets
    x = synth.normal_vector(int(off[-1]), 720, dtype=np.float32)
    zs = hs.matvec(_dev(x)).double().cpu().numpy()
    for c in range(H.HMX_TILE_CONFIGS):
        H.hmx_set_tile_config(hr.h, c)
        zr = hr.matvec(_dev(x)).double().cpu().numpy()
        assert _rel(zr, zs) <= 1e-6, c
    for q in range(len(pts)):
        a, b = off[q], off[q + 1]
        zd = orc.dense_matvec(pts[q], x[a:b], "gaussian", p0s[q])
        assert _rel(zr[a:b], zd) <= 1e-4
    hs.close()
    hr.close()
