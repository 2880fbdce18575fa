"""The caller's device allocator (hmx_params.dev_alloc / dev_free): every
device buffer of a build and of the handle's later calls comes from it and
goes back to it exactly once, results are those of the library's own
allocator bit for bit, and a failing allocation at any point of the build
returns HMX_ERR_OOM, produces no handle and returns every buffer taken."""
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


KW = dict(compute_dtype="f32", leaf_size=64, eta=1.5, aca_eps=1e-5, max_rank=32, sigma2=1e-1)


def test_hooks_serve_every_buffer_and_match(H):
    n = 20000
    pts = _dev(synth.uniform_points(n, 2, 601, dtype=np.float32))
    x = _dev(synth.normal_vector(n, 602, dtype=np.float32))
    a = H.TorchAllocator()
    print("build: N=%d FP32 with the caller's allocator" % n, flush=True)
    hu = H.HMatrix(pts, "gaussian", 0.01, allocator=a, **KW)
    st = hu.stats()
    print("allocations %d, outstanding %d bytes, handle holds %d bytes" % (
        a.allocs, a.outstanding_bytes, st.device_bytes), flush=True)
    assert a.allocs > 20
    assert a.outstanding_bytes == st.device_bytes  # the handle's buffers, nothing else
    hl = H.HMatrix(pts, "gaussian", 0.01, **KW)
    assert torch.equal(hu.matvec(x), hl.matvec(x))
    # later calls of the handle allocate through the hooks as well
    before = a.allocs
    c1 = torch.zeros_like(x)
    c2 = torch.zeros_like(x)
    s1 = H.hmx_cg_solve(hu.h, x, c1, rel_tol=1e-5, max_iter=500)
    s2 = H.hmx_cg_solve(hl.h, x, c2, rel_tol=1e-5, max_iter=500)
    assert s1 == s2 and torch.equal(c1, c2)
    H.hmx_autotune(hu.h, 1)
    assert a.allocs >= before + 7  # CG: 5 work buffers; autotune: 2 vectors
    assert a.outstanding_bytes == st.device_bytes
    hu.close()
    hl.close()
    assert a.outstanding_bytes == 0 and a.allocs == a.frees


class FailingAllocator:
    """TorchAllocator that returns NULL at its fail_at-th request."""

    def __init__(self, H, fail_at):
        self.inner = H.TorchAllocator()
        self.fail_at = fail_at
        take = self.inner.take

        def failing_take(nbytes):
            if self.inner.allocs == self.fail_at:
                return None
            return take(nbytes)
        self.inner.take = failing_take
        self.alloc_fn, self.free_fn = self.inner.alloc_fn, self.inner.free_fn


@pytest.mark.parametrize("symmetric", [0, 1])
def test_oom_at_every_stage_returns_everything(H, symmetric):
    n = 20000
    pts = _dev(synth.uniform_points(n, 3, 603, dtype=np.float32))
    probe = H.TorchAllocator()
    H.HMatrix(pts, "gaussian", 0.02, allocator=probe, symmetric_far=symmetric, **KW).close()
    total = probe.allocs
    print("a full build takes %d allocations" % total, flush=True)
    assert probe.outstanding_bytes == 0 and probe.frees == total
    picks = sorted(set([1, 2, 3, total // 4, total // 2, 3 * total // 4, total - 1, total]))
    for k in picks:
        fa = FailingAllocator(H, k)
        with pytest.raises(H.HmxError) as ei:
            H.HMatrix(pts, "gaussian", 0.02, allocator=fa, symmetric_far=symmetric, **KW)
        inner = fa.inner
        print("fail at allocation %d of %d: status %d, %d taken, %d returned, %d bytes left"
              % (k, total, ei.value.status, inner.allocs - 1, inner.frees,
                 inner.outstanding_bytes), flush=True)
        assert ei.value.status == H.HMX_ERR_OOM
        assert "allocator returned NULL" in str(ei.value)
        assert inner.allocs == k  # the build stopped at the failing request
        assert inner.outstanding_bytes == 0 and inner.frees == k - 1
    # the library still builds normally afterwards
    h = H.HMatrix(pts, "gaussian", 0.02, symmetric_far=symmetric, **KW)
    h.close()
