"""hipGraph-captured matvecs and the row-tile autotuner.

Graph replays must reproduce the eager matvecs bit for bit, replay after
replay with other work in between; every row-tile configuration the tuner
may choose must give the matvec within rounding of the default one.
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


@pytest.fixture(scope="module")
def hm(H):
    pts = synth.uniform_points(30000, 2, 900, dtype=np.float32)
    h = H.HMatrix(_dev(pts), "gaussian", 0.01, compute_dtype="f32", leaf_size=128, eta=1.5,
                  aca_eps=1e-5, max_rank=32, sigma2=0.5)
    yield h
    h.close()


def test_graph_replays_equal_eager(H, hm):
    x = _dev(synth.normal_vector(hm.n, 901, dtype=np.float32))
    ref = hm.matvec(x)
    z = torch.zeros_like(x)
    g = H.hmx_matvec_graph(hm.h, x, z)
    other = _dev(synth.normal_vector(hm.n, 902, dtype=np.float32))
    for rep in range(4):
        z.zero_()
        H.hmx_graph_launch(g)
        torch.cuda.synchronize()
        assert torch.equal(z, ref), rep
        hm.matvec(other)  # eager work on the same handle between replays
        torch.cuda.synchronize()
    H.hmx_graph_destroy(g)


def test_graph_with_accumulation(H, hm):
    x = _dev(synth.normal_vector(hm.n, 903, dtype=np.float32))
    ze = torch.zeros_like(x)
    for _ in range(3):
        hm.matvec(x, ze, alpha=0.5, beta=1.0)
    zg = torch.zeros_like(x)
    g = H.hmx_matvec_graph(hm.h, x, zg, alpha=0.5, beta=1.0, reps=3)
    H.hmx_graph_launch(g)
    torch.cuda.synchronize()
    assert torch.equal(zg, ze)
    H.hmx_graph_launch(g)  # three more
    for _ in range(3):
        hm.matvec(x, ze, alpha=0.5, beta=1.0)
    torch.cuda.synchronize()
    assert torch.equal(zg, ze)
    H.hmx_graph_destroy(g)


def test_autotune_configs_agree(H, hm):
    x = _dev(synth.normal_vector(hm.n, 904, dtype=np.float32))
    H.hmx_set_tile_config(hm.h, -1)
    ref = hm.matvec(x).double()
    for c in range(H.HMX_TILE_CONFIGS):
        H.hmx_set_tile_config(hm.h, c)
        z = hm.matvec(x).double()
        dev = (torch.linalg.norm(z - ref) / torch.linalg.norm(ref)).item()
        assert dev <= 1e-6, (c, dev)
        assert hm.stats().tile_config == c
    choice, times = H.hmx_autotune(hm.h, reps=3)
    print("autotune choice %d, ms per config %s" % (choice, np.round(times, 4)))
    assert 0 <= choice < H.HMX_TILE_CONFIGS and np.all(times > 0)
    assert times[choice] == times.min()
    assert hm.stats().tile_config == choice
    H.hmx_set_tile_config(hm.h, -1)
    assert torch.equal(hm.matvec(x).double(), ref)
    with pytest.raises(H.HmxError):
        H.hmx_set_tile_config(hm.h, H.HMX_TILE_CONFIGS)
