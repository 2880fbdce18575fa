"""Pins for the oracle's ordering step: global box, Morton codes (Section 4.4,
Algorithm 6) and the stable sort.  CPU only."""
import os
from fractions import Fraction

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "morton_examples.txt")


def _golden_groups():
    groups = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            parts = line.split()
            d = int(parts[0])
            xs = [float(Fraction(p)) for p in parts[1:1 + d]]
            code = int(parts[1 + d], 16)
            groups.setdefault(d, []).append((xs, code))
    return groups


@pytest.mark.parametrize("d", [1, 2, 3])
def test_morton_worked_examples(orc, d):
    rows = _golden_groups()[d]
    pts = np.array([r[0] for r in rows], dtype=np.float64)
    want = np.array([r[1] for r in rows], dtype=np.uint64)
    lo, hi = orc.global_box(pts)
    assert np.all(lo == 0.0) and np.all(hi == 1.0)
    got = orc.morton(pts)
    assert [hex(int(c)) for c in got] == [hex(int(c)) for c in want]


def _z_enumeration(cells, d, k):
    """Brute-force recursive enumeration of a 2^k-per-side grid in Z order:
    visit the 2^d half-size sub-cubes with dimension 0 as the most significant
    choice, recursing on the next lower coordinate bit."""
    if k == 0 or len(cells) <= 1:
        return list(cells)
    out = []
    for sub in range(1 << d):
        bits = [(sub >> (d - 1 - dim)) & 1 for dim in range(d)]
        part = [c for c in cells
                if all(((c[dim] >> (k - 1)) & 1) == bits[dim] for dim in range(d))]
        out.extend(_z_enumeration(part, d, k - 1))
    return out


@pytest.mark.parametrize("d,k", [(2, 3), (2, 4), (3, 2), (1, 5)])
def test_morton_grid_is_recursive_z_order(orc, d, k):
    side = 1 << k
    grid = np.stack(np.meshgrid(*[np.arange(side)] * d, indexing="ij"), -1).reshape(-1, d)
    rng = np.random.default_rng(5)
    grid = grid[rng.permutation(len(grid))]
    # cell corners i / 2^k plus the point (1,..,1) so the global box is [0,1]^d
    pts = np.vstack([grid / side, np.ones((1, d))])
    perm = orc.sort(orc.morton(pts))
    assert perm[-1] == len(grid)  # the clamped corner sorts last
    got = [tuple(grid[i]) for i in perm[:-1]]
    want = _z_enumeration([tuple(c) for c in grid], d, k)
    assert got == want


def test_global_box_matches_numpy(orc):
    p = synth.uniform_points(5000, 3, 1)
    lo, hi = orc.global_box(p)
    assert np.array_equal(lo, p.min(0)) and np.array_equal(hi, p.max(0))


def test_sort_is_stable_permutation(orc):
    p = synth.uniform_points(20000, 2, 2)
    p = np.vstack([p, p[:500]])  # duplicates -> equal codes
    codes = orc.morton(p)
    perm = orc.sort(codes)
    assert np.array_equal(np.sort(perm), np.arange(len(p)))
    assert np.array_equal(perm, np.argsort(codes, kind="stable"))
    sc = codes[perm]
    assert np.all(sc[1:] >= sc[:-1])
    # ties keep the original index order
    eq = sc[1:] == sc[:-1]
    assert eq.sum() >= 500 and np.all(perm[1:][eq] > perm[:-1][eq])


def test_degenerate_dimension_gets_zero_bits(orc):
    p = synth.uniform_points(100, 2, 3)
    p[:, 1] = 0.25  # zero extent in dimension 1
    codes = orc.morton(p)
    # dimension 1 occupies the even bit positions for d = 2
    assert np.all((codes & np.uint64(0x5555555555555555)) == 0)


def test_float32_inputs_promote_exactly(orc):
    p32 = synth.uniform_points(1000, 3, 4, dtype=np.float32)
    c1 = orc.morton(p32.astype(np.float64))
    lo, hi = orc.global_box(p32.astype(np.float64))
    assert lo.dtype == np.float64 and np.all(lo == p32.min(0).astype(np.float64))
    assert c1.dtype == np.uint64


def test_ordered_coords(orc):
    p = synth.uniform_points(777, 3, 6)
    codes, perm, soa = orc.order(p)
    assert np.array_equal(soa, p[perm].T)


def test_halton_points_first_terms():
    """Radical inverses: index 1..4 in base 2 are 1/2, 1/4, 3/4, 1/8; in base
    3 1/3, 2/3, 1/9, 4/9; in base 5 1/5, 2/5, 3/5, 4/5."""
    import synth
    p = synth.halton_points(4, 3)
    want = np.array([[1 / 2, 1 / 3, 1 / 5], [1 / 4, 2 / 3, 2 / 5], [3 / 4, 1 / 9, 3 / 5],
                     [1 / 8, 4 / 9, 4 / 5]])
    assert np.allclose(p, want, rtol=0, atol=4e-16)
    q = synth.halton_points(4096, 2)
    assert q.min() > 0 and q.max() < 1 and len(np.unique(q[:, 0])) == 4096
