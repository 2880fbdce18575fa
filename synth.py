"""Seeded synthetic inputs shared by the tests, the bench and the smoke check.

This module draws random numbers only.  It holds none of the H-matrix
method's arithmetic (no kernel, no ordering, no approximation), so both the
HIP path and the CPU oracle can consume its arrays without sharing code.

Every generator uses ``numpy.random.Generator(PCG64(seed))`` in float64 and
casts to the requested dtype at the end, so the two sides receive identical
bits.  The point distributions follow the workloads used in the paper's
results section (points in the unit square / cube) and the synthetic point
clouds this project measures on:

* uniform i.i.d. points in [0,1)^d,
* the Halton sequence (deterministic low-discrepancy points) in [0,1)^d,
* a Gaussian mixture in [0,1]^d (rejection of out-of-cube samples),
* standard-normal right-hand sides x,
* the regression target y = sin(2 pi p0) p1 + 0.01 xi of the kernel ridge
  regression workload.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def uniform_points(n: int, d: int, seed: int, dtype=np.float64) -> np.ndarray:
    """n points i.i.d. uniform in [0,1)^d, row-major (n, d)."""
    g = rng(seed)
    return np.ascontiguousarray(g.random((int(n), int(d)), dtype=np.float64).astype(dtype))


def gmm_points(n: int, d: int, seed: int, ncomp: int = 32, std_lo: float = 0.02,
               std_hi: float = 0.1, dtype=np.float64) -> np.ndarray:
    """n points from an equal-weight isotropic Gaussian mixture inside [0,1]^d.

    Means are uniform in [0.1, 0.9]^d, standard deviations uniform in
    [std_lo, std_hi].  Samples outside the unit cube are redrawn.
    """
    g = rng(seed)
    means = 0.1 + 0.8 * g.random((ncomp, d))
    stds = std_lo + (std_hi - std_lo) * g.random(ncomp)
    out = np.empty((int(n), int(d)), dtype=np.float64)
    filled = 0
    while filled < n:
        want = int((n - filled) * 1.3) + 16
        comp = g.integers(0, ncomp, size=want)
        p = means[comp] + stds[comp, None] * g.standard_normal((want, d))
        ok = np.all((p >= 0.0) & (p <= 1.0), axis=1)
        p = p[ok][: n - filled]
        out[filled: filled + len(p)] = p
        filled += len(p)
    return np.ascontiguousarray(out.astype(dtype))


def halton_points(n: int, d: int, start: int = 1, dtype=np.float64) -> np.ndarray:
    """The first n points of the Halton sequence in [0,1)^d (the point sets of
    the paper's model problem, Section 6.2): coordinate k of point i is the
    radical inverse of the index start + i in the k-th prime base (2, 3, 5),
    i.e. the base-b digits of the index mirrored at the radix point.  The
    default start 1 skips the origin."""
    bases = (2, 3, 5)[: int(d)]
    idx = np.arange(int(start), int(start) + int(n), dtype=np.int64)
    out = np.empty((int(n), int(d)), dtype=np.float64)
    for k, b in enumerate(bases):
        v = np.zeros(int(n), dtype=np.float64)
        f = 1.0 / b
        i = idx.copy()
        while np.any(i > 0):
            v += f * (i % b)
            i //= b
            f /= b
        out[:, k] = v
    return np.ascontiguousarray(out.astype(dtype))


def normal_vector(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """x ~ N(0, I_n)."""
    g = rng(seed)
    return g.standard_normal(int(n)).astype(dtype)


def krr_target(points: np.ndarray, seed: int, noise: float = 0.01, dtype=np.float64) -> np.ndarray:
    """y = sin(2 pi p0) * p1 + noise * xi with xi ~ N(0,1)."""
    g = rng(seed)
    p = np.asarray(points, dtype=np.float64)
    xi = g.standard_normal(p.shape[0])
    return (np.sin(2.0 * np.pi * p[:, 0]) * p[:, 1] + noise * xi).astype(dtype)


def log_uniform(lo: float, hi: float, size, seed: int) -> np.ndarray:
    g = rng(seed)
    return np.exp(np.log(lo) + (np.log(hi) - np.log(lo)) * g.random(size))


def sample_rows(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct row indices in [0, n), sorted."""
    g = rng(seed)
    k = min(int(k), int(n))
    return np.sort(g.choice(int(n), size=k, replace=False)).astype(np.int64)


# Rank-predictor layer sizes (input, three hidden layers, output) and the
# packing order of its parameters: W1, b1, W2, b2, W3, b3, W4, b4.
MLP_LAYERS = (8, 64, 64, 64, 1)


def mlp_init_params(seed: int) -> np.ndarray:
    """Initial predictor weights: W ~ N(0, 2 / fan_in) (He), biases 0, float32."""
    g = rng(seed)
    parts = []
    for fan_in, fan_out in zip(MLP_LAYERS[:-1], MLP_LAYERS[1:]):
        parts.append(g.standard_normal(fan_out * fan_in) * np.sqrt(2.0 / fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def batch_indices(n: int, batch: int, steps: int, seed: int) -> np.ndarray:
    """steps x batch sample indices, each step an independent draw without
    replacement from [0, n) (with replacement when batch > n), int64."""
    g = rng(seed)
    out = np.empty((int(steps), int(batch)), np.int64)
    for s in range(int(steps)):
        out[s] = g.choice(int(n), size=int(batch), replace=int(batch) > int(n))
    return out.reshape(-1)


# Workload recipes (sizes, kernels, seeds).  Plain data, no arithmetic.
WORKLOADS = {
    # small plain FP64 case, checked against the dense product
    "gauss2d_n4096_f64": dict(n=4096, d=2, dist="uniform", pts_seed=11, x_seed=12,
                              kernel="gaussian", p0=0.1, leaf=64, eta=1.5, eps=1e-6,
                              kmax=32, dtype="f64"),
    # plain method on the GPU in FP32 at N = 2^20
    "gauss2d_n1m_f32": dict(n=1 << 20, d=2, dist="uniform", pts_seed=21, x_seed=2200,
                            kernel="gaussian", p0=0.01, leaf=256, eta=1.5, eps=1e-5,
                            kmax=64, dtype="f32", n_matvec=100, mixed_eps=3e-3,
                            cpu_rows_frac=1.0),
    # N = 2^22 points uniform in [0,1]^3, Gaussian p0 = the first draw of the
    # log-uniform [0.002, 0.05] evaluation draws (seed 52): the ACA up to the
    # factor pools (the stored pools exceed one GPU's memory)
    "gauss3d_n4m_aca": dict(n=1 << 22, d=3, dist="uniform", pts_seed=51, p0_seed=52,
                            p0_lo=0.002, p0_hi=0.05, kernel="gaussian", leaf=64, eta=1.5,
                            eps=1e-5, kmax=64, dtype="f32"),
    # the same with BF16 storage of the near field and the factors
    "gauss2d_n1m_bf16": dict(n=1 << 20, d=2, dist="uniform", pts_seed=21, x_seed=2200,
                             kernel="gaussian", p0=0.01, leaf=256, eta=1.5, eps=1e-5,
                             kmax=64, dtype="f32", storage="bf16", n_matvec=100),
}
