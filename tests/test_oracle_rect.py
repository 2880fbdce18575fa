"""Pins for the oracle's rectangular H-matrix A_{phi, Y1 x Y2} (the kernel
matrix between two point sets, Section 6): partition from the block
Y1 x Y2 by Algorithm 1 with eq. (3), each set ordered in its own box and
clustered in its own tree; the product against the brute-force dense
product.  CPU only."""
import math

import numpy as np
import pytest
from scipy.spatial.distance import cdist
from scipy.special import k1

import synth


def _dense_ref(p1, p2, x, kind, p0):
    """The dense product from scipy distances (an independent evaluation)."""
    d = p1.shape[1]
    r = cdist(p1, p2)
    if kind == "gaussian":
        A = np.exp(-r * r / p0)
    elif kind == "matern32":
        s = math.sqrt(3.0) * r / p0
        A = (1.0 + s) * np.exp(-s)
    else:
        beta = 1.0 + d / 2.0
        s = r / p0
        with np.errstate(invalid="ignore", divide="ignore"):
            A = np.where(s > 0, s * k1(np.where(s > 0, s, 1.0)), 1.0)
        A = A / (2.0 ** (beta - 1.0) * math.gamma(beta))
    return A @ x


@pytest.mark.parametrize("kind,p0,d", [("gaussian", 0.05, 2), ("matern32", 0.2, 3),
                                       ("matern_nu1", 0.3, 1), ("matern_nu1", 0.1, 3)])
def test_dense_rect_matches_scipy(orc, kind, p0, d):
    p1 = synth.uniform_points(300, d, 1)
    p2 = synth.uniform_points(170, d, 2)
    x = synth.normal_vector(170, 3)
    z = orc.dense_matvec_rect(p1, p2, x, kind, p0)
    ref = _dense_ref(p1, p2, x, kind, p0)
    assert np.linalg.norm(z - ref) <= 1e-13 * np.linalg.norm(ref)


def _py_block_tree_rect(soa1, soa2, leaf, eta):
    """Algorithm 1 from the block (Y1, Y2), written independently in Python
    with the unsquared admissibility and the floor-half cluster split."""
    out_adm, out_dense = set(), set()

    def box(soa, a, b):
        seg = soa[:, a:b]
        return seg.min(1), seg.max(1)

    def adm(t, s):
        at, bt = box(soa1, *t)
        as_, bs = box(soa2, *s)
        diam_t = math.sqrt(sum((bt - at) ** 2))
        diam_s = math.sqrt(sum((bs - as_) ** 2))
        dist = math.sqrt(sum(max(0.0, at[i] - bs[i]) ** 2 + max(0.0, as_[i] - bt[i]) ** 2
                             for i in range(soa1.shape[0])))
        return min(diam_t, diam_s) <= eta * dist

    def kids(c):
        a, b = c
        m = a + (b - a) // 2
        return [(a, m), (m, b)]

    def rec(t, s):
        if adm(t, s):
            out_adm.add(t + s)
        elif t[1] - t[0] > leaf and s[1] - s[0] > leaf:
            for t2 in kids(t):
                for s2 in kids(s):
                    rec(t2, s2)
        else:
            out_dense.add(t + s)

    rec((0, soa1.shape[1]), (0, soa2.shape[1]))
    return out_adm, out_dense


@pytest.mark.parametrize("n1,n2,d,leaf,eta", [(600, 250, 2, 16, 1.5), (300, 900, 3, 20, 1.0),
                                               (513, 513, 2, 8, 2.5), (100, 700, 1, 4, 1.5)])
def test_partition_rect_equals_recursive_alg1(orc, n1, n2, d, leaf, eta):
    _, _, soa1 = orc.order(synth.uniform_points(n1, d, 10 + n1))
    # the second set in a shifted, stretched box: clusters of the two trees differ
    p2 = synth.uniform_points(n2, d, 20 + n2) * 1.5 + 0.3
    _, _, soa2 = orc.order(p2)
    adm, den, ls = orc.partition_rect(soa1, soa2, leaf, eta)
    pa, pd = _py_block_tree_rect(soa1, soa2, leaf, eta)
    assert set(map(tuple, adm[:, :4].tolist())) == pa
    assert set(map(tuple, den[:, :4].tolist())) == pd
    assert len(pa) == len(adm) and len(pd) == len(den)
    # every entry of Y1 x Y2 covered once
    cnt = np.zeros((n1, n2), np.int16)
    for r in np.vstack([adm, den]):
        cnt[r[0]:r[1], r[2]:r[3]] += 1
    assert np.all(cnt == 1)
    assert np.all(np.diff(adm[:, 4]) >= 0) and np.all(np.diff(den[:, 4]) >= 0)


def test_partition_rect_of_one_set_is_the_square_partition(orc):
    _, _, soa = orc.order(synth.uniform_points(1500, 2, 31))
    a1, d1, l1 = orc.partition(soa, 32, 1.5)
    a2, d2, l2 = orc.partition_rect(soa, soa, 32, 1.5)
    assert np.array_equal(a1, a2) and np.array_equal(d1, d2) and np.array_equal(l1, l2)


def test_hmvp_rect_reduces_to_dense(orc):
    p1 = synth.uniform_points(800, 2, 41)
    p2 = synth.uniform_points(600, 2, 42) + np.array([0.5, 0.0])
    x = synth.normal_vector(600, 43)
    ref = orc.dense_matvec_rect(p1, p2, x, "gaussian", 0.05)
    # eta = 0: no admissible block; leaf >= n: one dense block
    for leaf, eta in [(16, 0.0), (1000, 1.5)]:
        z, _, st = orc.hmvp_rect(p1, p2, x, "gaussian", 0.05, leaf, eta, 16, 1e-8)
        assert st["n_adm"] == 0
        assert np.linalg.norm(z - ref) <= 1e-13 * np.linalg.norm(ref)
    # ACA to full rank (eps = 0) is exact
    z, _, st = orc.hmvp_rect(p1, p2, x, "gaussian", 0.05, 16, 1.5, 128, 0.0)
    assert st["n_adm"] > 0
    assert np.linalg.norm(z - ref) <= 1e-11 * np.linalg.norm(ref)


def test_hmvp_rect_of_one_set_is_the_square_product(orc):
    p = synth.uniform_points(2000, 3, 51)
    x = synth.normal_vector(2000, 52)
    zs, rs, _ = orc.hmvp(p, x, "matern32", 0.2, 40, 1.5, 32, 1e-7, want_ranks=True)
    zr, rr, _ = orc.hmvp_rect(p, p, x, "matern32", 0.2, 40, 1.5, 32, 1e-7, want_ranks=True)
    assert np.array_equal(rs, rr)
    assert np.linalg.norm(zr - zs) <= 1e-14 * np.linalg.norm(zs)


@pytest.mark.parametrize("kind,p0", [("gaussian", 0.02), ("matern_nu1", 0.1)])
def test_hmvp_rect_error_and_algebra(orc, kind, p0):
    p1 = synth.uniform_points(3000, 2, 61)
    p2 = synth.uniform_points(1200, 2, 62) * 0.8
    x = synth.normal_vector(1200, 63)
    ref = orc.dense_matvec_rect(p1, p2, x, kind, p0)
    errs = []
    for eps in (1e-3, 1e-5, 1e-7):
        z, _, _ = orc.hmvp_rect(p1, p2, x, kind, p0, 32, 1.5, 64, eps)
        e = np.linalg.norm(z - ref) / np.linalg.norm(ref)
        assert e <= 10 * eps, (eps, e)
        errs.append(e)
    assert errs[0] > errs[1] > errs[2]
    z0 = synth.normal_vector(3000, 64)
    z1, _, _ = orc.hmvp_rect(p1, p2, x, kind, p0, 32, 1.5, 64, 1e-7)
    z2, _, _ = orc.hmvp_rect(p1, p2, x, kind, p0, 32, 1.5, 64, 1e-7, alpha=0.5, beta=-2.0,
                             z=z0)
    assert np.allclose(z2, 0.5 * z1 - 2.0 * z0, rtol=0, atol=1e-13 * np.abs(z1).max())
