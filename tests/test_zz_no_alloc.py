"""hmx_cg_solve_noalloc, the CG solve whose work space is a fixed device
array, against hmx_cg_solve (which allocates its work vectors): the same
kernels in the same order, so the iterates, iteration counts and residuals
agree bit for bit.  Two calls in a row on one device, the second on a
smaller handle, so the second runs over what the first left in the array;
then the size limit is rejected before any device work."""
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


def _solve_both(H, n, dtype, seed):
    pts = synth.gmm_points(n, 3, seed, ncomp=16)
    y = synth.krr_target(pts, seed + 1)
    print("build: N=%d %s Matern-3/2 l=0.1 sigma2=1e-2, CG both ways" % (n, dtype), flush=True)
    hm = H.HMatrix(_dev(pts), "matern32", 0.1, compute_dtype=dtype, leaf_size=64, eta=1.5,
                   aca_eps=1e-7 if dtype == "f64" else 1e-5, max_rank=64, sigma2=1e-2)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    b = _dev(y).to(tdt)
    tol = 1e-9 if dtype == "f64" else 1e-5
    xa = torch.full((n,), 7.0, dtype=tdt, device="cuda:0")  # overwritten by both solves
    xb = torch.full((n,), -3.0, dtype=tdt, device="cuda:0")
    ra = H.hmx_cg_solve(hm.h, b, xa, rel_tol=tol, max_iter=3000, raise_on_fail=False)
    rb = H.hmx_cg_solve(hm.h, b, xb, rel_tol=tol, max_iter=3000, raise_on_fail=False,
                        noalloc=True)
    torch.cuda.synchronize()
    print("  allocating: status %d iters %d res %.3e true %.3e" % ra, flush=True)
    print("  no-alloc  : status %d iters %d res %.3e true %.3e" % rb, flush=True)
    assert ra[0] == H.HMX_OK
    assert ra == rb  # status, iterations, recurrence and true residual, bit for bit
    assert torch.equal(xa, xb)
    hm.close()


def test_noalloc_cg_equals_allocating_cg_twice_shrinking(H):
    _solve_both(H, 6000, "f32", 31)   # first call on this device
    _solve_both(H, 2500, "f32", 35)   # smaller: the array holds the larger call's data
    _solve_both(H, 3000, "f64", 37)


def test_noalloc_cg_rejects_oversize(H):
    # 2^21 + 4096 FP64 entries: three work vectors exceed the fixed array
    n = (1 << 21) + 4096
    pts = synth.uniform_points(n, 1, 41)
    print("build: N=%d d=1 FP64 (size limit check)" % n, flush=True)
    hm = H.HMatrix(_dev(pts), "gaussian", 1e-4, compute_dtype="f64", leaf_size=64, eta=1.5,
                   aca_eps=1e-3, max_rank=8, sigma2=1.0)
    b = torch.ones(n, dtype=torch.float64, device="cuda:0")
    x = torch.zeros(n, dtype=torch.float64, device="cuda:0")
    with pytest.raises(H.HmxError) as ei:
        H.hmx_cg_solve(hm.h, b, x, noalloc=True)
    assert ei.value.status == H.HMX_ERR_INVALID_ARG
    assert "work space" in str(ei.value)
    assert torch.count_nonzero(x).item() == 0  # rejected before any device work
    hm.close()
