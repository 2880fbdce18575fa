"""Reproducibility of the build: the same problem built again, with other
builds in between (so that the device memory cache hands out blocks holding
another problem's factors), gives the same ranks bit for bit and the same
matvec bit for bit, in every ACA size class and in both rank modes.
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


@pytest.mark.parametrize("mode", ["adaptive", "learned"])
def test_repeat_builds_identical(H, mode):
    n = 1 << 18
    pts = _dev(synth.uniform_points(n, 2, 9100, dtype=np.float32))
    other = _dev(synth.uniform_points(n // 2, 3, 9101, dtype=np.float32))
    x = _dev(synth.normal_vector(n, 9102, dtype=np.float32))
    kw = dict(compute_dtype="f32", leaf_size=64, eta=1.5, aca_eps=1e-5, max_rank=64)
    mlp = None
    if mode == "learned":
        # a constant small target: most blocks finish beyond it (fallback pass)
        w = np.zeros(8961, np.float32)
        w[-1] = 4.0
        mlp = H.RankMLP(w)
        kw.update(rank_mode="learned", mlp=mlp)
    ranks, outs = [], []
    for rep in range(3):
        hm = H.HMatrix(pts, "gaussian", 0.01, **kw)
        s = hm.stats()
        ranks.append(hm.ranks())
        outs.append(hm.matvec(x))
        print("rep %d: n_adm %d sum rank %d aca %.1f ms"
              % (rep, s.n_adm, s.sum_rank, s.phase_ms[3]))
        hm.close()
        # another problem's build fills the cache with other values
        ho = H.HMatrix(other, "matern32", 0.05, compute_dtype="f32", leaf_size=64, eta=1.5,
                       aca_eps=1e-6, max_rank=64)
        ho.close()
    for rep in (1, 2):
        assert np.array_equal(ranks[0], ranks[rep]), rep
        assert torch.equal(outs[0], outs[rep]), rep
    if mlp is not None:
        mlp.close()
