"""Benchmark of the H-matrix hot path on one MI355X.

A step is one pass of the whole path over one synthetic point set: build
(ordering, cluster tree, block-tree traversal, rank prediction, batched ACA,
near field, matvec plan) followed by the workload's matvecs.  Two forms run
on the same points and vectors:

  plain         FP32 arithmetic and storage, adaptive ACA (k_max-sized
                scratch), stored near field;
  learned_mixed the rank predictor sizes every block's ACA storage (trained
                first, on the ranks of plain ACA builds of other point sets at
                the same tolerance), BF16 factors and near field (round to
                nearest even), FP32 arithmetic, FP64 ACA norm; its ACA
                tolerance is the workload's mixed_eps, chosen so that the
                ACA's own error is about the BF16 rounding error of the
                stored entries (a smaller one buys little accuracy, a
                larger one dominates);

and a third, plain_eq, is the plain form with the ACA tolerance raised until
its matvec error matches learned_mixed's (equal relative error).  Errors are
measured on sampled rows against an FP64 dense product computed with plain
PyTorch on the GPU.  The printed line's value is the learned_mixed form's
H-matvec throughput in algorithmic GB/s (stored near field and factors read
once, x / z / permutation once, t written and read); the timed steps are its
steps.  Each form's row-tile shape is picked once by the library's autotuner
(hmx_autotune, on the warm-up build).  The roofline is the row-tile matvec kernel's, timed live with HIP
events on the stream it runs on; cpu_baseline is the oracle timed on a
bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--matvecs M]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "H-build seconds + H-matvec GB/s at N=2^22, learned/mixed vs plain, equal rel err"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
FP32_PEAK = 157.3e12   # MI355X FP32 vector FLOP/s
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "rowtile_traffic.json")

# the forms compared (hmx_params overrides on top of the workload's settings)
FORMS = {
    "plain_f64": dict(compute_dtype="f64", storage_dtype="f64", near_dtype="f64",
                      rank_mode="adaptive"),
    "plain": dict(storage_dtype="f32", near_dtype="f32", rank_mode="adaptive"),
    "learned_mixed": dict(storage_dtype="bf16", near_dtype="bf16", rank_mode="learned"),
}
# predictor training recipe: plain ACA-only builds of other point sets
TRAIN = dict(builds=24, log2n_lo=14, log2n_hi=18, p0_lo=0.002, p0_hi=0.05, seed=5300,
             steps=800, batch=2048, lr=3e-3, q=0.9)


def kernel_source_hash(text=None) -> str:
    """Hash of the row-tile kernel's source: the storage decoders it reads the
    pools with and the phase-2 section of k_mvp.hip up to the end of its
    launcher (the counters stay valid while this text is unchanged)."""
    if text is None:
        with open(os.path.join(ROOT, "paper_1708_09707_amd", "csrc", "k_mvp.hip")) as f:
            text = f.read()
    a = text.index("template <typename S, typename T>\nstruct Dec;")
    b = text.index("\n", text.index("__device__ __forceinline__ u32x4 nt_load("))
    c = text.index("// phase 2: one workgroup per row tile")
    d = text.index("}  // namespace", text.index("hipError_t rowtile_dispatch("))
    return hashlib.sha256((text[a:b] + text[c:d]).encode()).hexdigest()[:16]


def rowtile_bytes(st, esz=4) -> float:
    """Algorithmic bytes of one row-tile launch: the stored near field and U
    read once, t read once, z written once, the permutation read once
    (esz: bytes per vector entry, 8 for FP64 arithmetic).  Re-reads of
    x|sigma segments served from cache are not counted."""
    return (st.near_entries * st.near_entry_bytes + st.u_entries * st.entry_bytes
            + st.sum_rank * esz + st.n * (esz + 4))


# row-tile shapes (lanes per row group, row vectors per lane) of configurations
# c = mode * 5 + shape
ROWTILE_SHAPES = ((16, 1), (32, 1), (64, 1), (64, 2), (64, 4), (8, 1))


def measured_traffic(workload: str, form: str, config: int):
    """HBM bytes per row-tile launch of the chosen configuration's kernel
    shape, from the committed rocprofv3 counter summary, if it was taken on
    the current kernel source and this form."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if (rec.get("kernel_source") != kernel_source_hash() or rec.get("workload") != workload
            or rec.get("form") != form or config is None or config < 0):
        return None
    L, RV = ROWTILE_SHAPES[config % 5 if config < 15 else 5]
    return rec.get("bytes_per_launch_by_shape", {}).get("%d,%d" % (L, RV))


# ACA tolerances tried for the plain form at equal error (errors grow with
# eps; the grid is fine where the learned form's errors lie)
EQ_GRID = (3e-5, 1e-4, 3e-4, 1e-3, 2e-3, 3e-3, 4e-3, 5e-3, 7e-3, 1e-2)


def dense_rows_fp64(torch, pts_d, x_d, p0, rows_d):
    """z[rows] of the FP64 dense product exp(-|y_i - y_j|^2 / p0) x, plain
    PyTorch on the GPU (an independent reference for the error)."""
    P = pts_d.double()
    x = x_d.double()
    ref = torch.zeros(rows_d.numel(), dtype=torch.float64, device=P.device)
    step = 1 << 16
    for c0 in range(0, P.shape[0], step):
        d2 = ((P[rows_d, None, :] - P[None, c0:c0 + step, :]) ** 2).sum(-1)
        ref += torch.exp(-d2 / p0) @ x[c0:c0 + step]
    return ref


def train_predictor(torch, H, wl, eps, log, d=None):
    """Train the rank predictor on (features, rank) pairs of plain ACA-only
    builds at tolerance eps (in d dimensions); returns (RankMLP, info)."""
    d = wl["d"] if d is None else d
    t0 = time.perf_counter()
    g = synth.rng(TRAIN["seed"])
    nb = TRAIN["builds"]
    ns = np.round(2.0 ** (TRAIN["log2n_lo"] + (TRAIN["log2n_hi"] - TRAIN["log2n_lo"])
                          * g.random(nb))).astype(int)
    p0s = synth.log_uniform(TRAIN["p0_lo"], TRAIN["p0_hi"], nb, TRAIN["seed"] + 1)
    Xs, ys = [], []
    for b in range(nb):
        pts = synth.uniform_points(int(ns[b]), d, TRAIN["seed"] + 10 + b, dtype=np.float32)
        hm = H.HMatrix(torch.from_numpy(pts).cuda(), wl["kernel"], float(p0s[b]),
                       compute_dtype="f32", leaf_size=wl["leaf"], eta=wl["eta"],
                       aca_eps=eps, max_rank=wl["kmax"], aca_only=1)
        F, y = H.hmx_block_features(hm.h)
        Xs.append(F.clone())
        ys.append(y.clone())
        hm.close()
    X = torch.cat(Xs)
    y = torch.cat(ys)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    mlp = H.RankMLP(synth.mlp_init_params(TRAIN["seed"] + 2))
    mlp.fit_normalization(X)
    idx = torch.from_numpy(synth.batch_indices(X.shape[0], TRAIN["batch"], TRAIN["steps"],
                                               TRAIN["seed"] + 3)).cuda()
    losses = torch.zeros(TRAIN["steps"], dtype=torch.float64, device="cuda")
    mlp.train(X, y, idx, TRAIN["batch"], TRAIN["steps"], q=TRAIN["q"], lr=TRAIN["lr"],
              losses=losses)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    lh = losses.cpu().numpy()
    info = {"pairs": int(X.shape[0]), "builds": nb, "data_s": t1 - t0, "train_s": t2 - t1,
            "steps": TRAIN["steps"], "batch": TRAIN["batch"], "quantile": TRAIN["q"],
            "loss_first": float(lh[:20].mean()), "loss_last": float(lh[-20:].mean())}
    log("bench: predictor trained on %d pairs from %d builds (%.2f s data, %.2f s training), "
        "loss %.3f -> %.3f" % (info["pairs"], nb, info["data_s"], info["train_s"],
                               info["loss_first"], info["loss_last"]))
    return mlp, info


def n22_aca_builds(torch, H, log, full=True, one_shot=False):
    """Builds up to the ACA at N = 2^22 in 3-d (the stored pools exceed one
    GPU): plain (k_max-sized ACA scratch, in chunks) against learned sizing
    (sizing form: identical ranks, storage from the predictor) and the
    one-shot learned form (the predicted steps without the per-step test)."""
    wl = dict(synth.WORKLOADS["gauss3d_n4m_aca"])
    p0 = float(synth.log_uniform(wl["p0_lo"], wl["p0_hi"], 5, wl["p0_seed"])[0])
    pts = synth.uniform_points(wl["n"], 3, wl["pts_seed"], dtype=np.float32)
    pts_d = torch.from_numpy(pts).cuda()
    mlp, info = train_predictor(torch, H, wl, wl["eps"], log, d=3)
    res = {"workload": "gauss3d_n4m_aca: N=%d uniform in [0,1]^3, gaussian p0=%.5g, leaf %d, "
                       "eta %g, ACA eps %g, max rank %d, FP32; build up to the ACA" % (
                           wl["n"], p0, wl["leaf"], wl["eta"], wl["eps"], wl["kmax"]),
           "predictor_training": info}
    ranks = {}
    # two builds per form, interleaved: the first build of the process also
    # pays the first touch of the device memory it takes into the cache
    for rep in range(2):
        for form in ("plain", "learned") + (("learned_one_shot",) if one_shot else ()):
            kw = {"plain": {}, "learned": dict(rank_mode="learned", mlp=mlp),
                  "learned_one_shot": dict(rank_mode="learned", mlp=mlp, learned_one_shot=1)}[form]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            hm = H.HMatrix(pts_d, wl["kernel"], p0, compute_dtype="f32", leaf_size=wl["leaf"],
                           eta=wl["eta"], aca_eps=wl["eps"], max_rank=wl["kmax"], aca_only=1,
                           **kw)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st = hm.stats()
            if rep == 0:
                ranks[form] = hm.ranks()
            else:
                assert np.array_equal(ranks[form], hm.ranks()), "repeat build differs"
            r = res.setdefault(form, {"build_s_each": [], "phase_ms_each": []})
            r["build_s_each"].append(t1 - t0)
            r["phase_ms_each"].append(list(st.phase_ms))
            r.update({"build_s": min(r["build_s_each"]), "aca_chunks": st.aca_chunks,
                      "aca_capacity_entries": st.aca_capacity, "aca_fallback": st.aca_fallback,
                      "aca_overflow": st.aca_overflow,
                      "predict_ms": st.predict_ms, "n_adm": st.n_adm, "n_dense": st.n_dense,
                      "sum_rank": st.sum_rank})
            r["aca_ms"] = min(ph[3] for ph in r["phase_ms_each"])
            log("bench: 2^22 3-d %s #%d: build %.2f s (ACA %.2f s in %d chunks, capacity %.3g "
                "entries, %d fallbacks; phases %s)"
                % (form, rep, t1 - t0, st.phase_ms[3] / 1e3, st.aca_chunks, st.aca_capacity,
                   st.aca_fallback, " ".join("%.0f" % v for v in st.phase_ms[:6])))
            hm.close()
    res["ranks_identical"] = bool(np.array_equal(ranks["plain"], ranks["learned"]))
    res["build_speedup"] = res["plain"]["build_s"] / res["learned"]["build_s"]
    if one_shot:
        # one-shot: exactly the predicted steps, then the test on the last term
        # (adaptive continuation on failure), so every block still meets the
        # tolerance; ranks may exceed the adaptive ones
        res["one_shot_build_speedup"] = (res["plain"]["build_s"]
                                         / res["learned_one_shot"]["build_s"])
        res["one_shot_sum_rank_ratio"] = (float(np.sum(ranks["learned_one_shot"]))
                                          / max(float(np.sum(ranks["plain"])), 1.0))
    H.hmx_trim()
    torch.cuda.empty_cache()
    if full:
        res["learned_mixed_full"] = n22_full_path(torch, H, log, wl, pts_d, p0, mlp)
    mlp.close()
    H.hmx_trim()
    return res


def n22_full_path(torch, H, log, wl, pts_d, p0, mlp, eps=3e-3, M=10, nrows=1024):
    """The whole path at N = 2^22 in 3-d for the learned / mixed-precision
    form: learned sizing, BF16 factors and near field, the symmetric far
    field (each factor pair stored once).  Build time, matvec time and bytes,
    and the product's error on sampled rows against an FP64 dense product.
    (The plain FP32 form at this tolerance does not fit one GPU, even with its
    near field evaluated in the product: its 153 GB of factors are held twice
    while the build lays them out tile-major.)"""
    n = wl["n"]
    kw = dict(compute_dtype="f32", storage_dtype="bf16", leaf_size=wl["leaf"], eta=wl["eta"],
              aca_eps=eps, max_rank=wl["kmax"], rank_mode="learned", mlp=mlp, symmetric_far=1)
    times, fresh = [], []
    for rep in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hm = H.HMatrix(pts_d, wl["kernel"], p0, **kw)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        st = hm.stats()
        fresh.append(st.alloc_fresh_bytes)
        if rep == 0:
            hm.close()
    # the first build's blocks the second did not take (its ACA scratch peak)
    # go back to the driver, so torch has room for the reference rows
    H.hmx_trim()
    stream = torch.cuda.current_stream()
    H.hmx_autotune(hm.h, 2, stream)
    x = torch.from_numpy(synth.normal_vector(n, 5400, dtype=np.float32)).cuda()
    z = torch.empty_like(x)
    g = H.hmx_matvec_graph(hm.h, x, z)
    H.hmx_graph_launch(g, stream)
    H.hmx_profile_begin(hm.h, 3)
    for _ in range(3):
        H.hmx_matvec(hm.h, x, z, 1.0, 0.0, stream)
    phase_ms, calls = H.hmx_profile_end(hm.h)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(M):
        H.hmx_graph_launch(g, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    mv_ms = e0.elapsed_time(e1) / M
    H.hmx_graph_destroy(g)
    rows_d = torch.from_numpy(synth.sample_rows(n, nrows, 5401)).cuda()
    ref = dense_rows_fp64(torch, pts_d, x, p0, rows_d)
    err = (torch.linalg.norm(z.double()[rows_d] - ref) / torch.linalg.norm(ref)).item()
    fb = (st.u_entries + st.v_entries) * st.entry_bytes
    out = {"eps": eps, "build_s_each": times, "build_s": min(times),
           "build_fresh_bytes_each": fresh,
           "matvec_bytes": st.matvec_bytes, "matvec_gbs": st.matvec_bytes / (mv_ms * 1e-3) / 1e9,
           "build_phase_ms": list(st.phase_ms), "sum_rank": st.sum_rank,
           "factor_entries": st.factor_entries, "near_entries": st.near_entries,
           "device_bytes": st.device_bytes, "aca_overflow": st.aca_overflow,
           "aca_fallback": st.aca_fallback, "matvec_ms": mv_ms,
           "matvec_phase_ms": list(phase_ms / max(calls, 1)),
           "factor_bytes_read_per_matvec": fb, "factor_gbs": fb / (mv_ms * 1e-3) / 1e9,
           "near_evals_per_s": st.near_entries / (mv_ms * 1e-3), "rel_err_rows": err,
           "rows": nrows}
    log("bench: 2^22 3-d learned/mixed full path: build %.2f s, device %.1f GB, matvec %.2f ms "
        "(%.3g B, %.0f GB/s), rel err %.2e"
        % (out["build_s"], st.device_bytes / 1e9, mv_ms, st.matvec_bytes, out["matvec_gbs"],
           err))
    hm.close()
    return out


def np_leg(torch, H, log, n, d, kw, p0=1.0, reps=2, nrows=256, forms=("np", "p", "stored"),
           points="halton", seed=0):
    """Build and matvec times of the far field without precomputation (np: ACA
    and near field recomputed in every product), with stored factors and a
    recomputed near field (p: the paper's precomputed mode, whose dense blocks
    are never stored) and with everything stored; the products' error on
    sampled rows against an FP64 dense product (Gaussian exp(-r^2 / p0))."""
    if points == "halton":
        pts = synth.halton_points(n, d)
    else:
        pts = synth.uniform_points(n, d, seed)
    dt = torch.float64 if kw.get("compute_dtype") == "f64" else torch.float32
    pts_d = torch.from_numpy(pts).cuda().to(dt)
    x = torch.from_numpy(synth.normal_vector(n, 7100)).cuda().to(dt)
    z = torch.empty_like(x)
    rows_d = torch.from_numpy(synth.sample_rows(n, nrows, 7101)).cuda()
    ref = dense_rows_fp64(torch, pts_d, x, p0, rows_d)
    out = {}
    for form in forms:
        extra = {"np": dict(far_recompute=1, near_recompute=1),
                 "p": dict(near_recompute=1), "stored": {}}[form]
        H.hmx_trim()
        times = []
        for rep in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            hm = H.HMatrix(pts_d, "gaussian", p0, **kw, **extra)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            if rep + 1 < reps:
                hm.close()
        st = hm.stats()
        mv = []
        for rep in range(reps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            H.hmx_matvec(hm.h, x, z)
            torch.cuda.synchronize()
            mv.append(time.perf_counter() - t0)
        err = (torch.linalg.norm(z.double()[rows_d] - ref) / torch.linalg.norm(ref)).item()
        st2 = hm.stats()
        out[form] = {"build_s_each": times, "build_s": min(times), "matvec_s_each": mv,
                     "matvec_s": min(mv[1:]), "rel_err_rows": err, "n_adm": st.n_adm,
                     "n_dense": st.n_dense, "sum_rank": st2.sum_rank, "aca_chunks": st.aca_chunks,
                     "near_entries": st.near_entries, "device_bytes": st.device_bytes}
        log("bench: N=%d d=%d %s: build %.3f s, matvec %.3f s, rel err %.2e, device %.2f GB, "
            "%d chunks" % (n, d, form, min(times), min(mv[1:]), err, st.device_bytes / 1e9,
                           st.aca_chunks))
        hm.close()
    return out


def dense_rows_matern32(torch, pts_d, x_d, ell, rows_d):
    """z[rows] of the FP64 dense Matern-3/2 product (plain PyTorch on the GPU)."""
    P = pts_d.double()
    x = x_d.double()
    ref = torch.zeros(rows_d.numel(), dtype=torch.float64, device=P.device)
    step = 1 << 15
    s3 = np.sqrt(3.0) / ell
    for c0 in range(0, P.shape[0], step):
        r = torch.sqrt(((P[rows_d, None, :] - P[None, c0:c0 + step, :]) ** 2).sum(-1)) * s3
        ref += ((1.0 + r) * torch.exp(-r)) @ x[c0:c0 + step]
    return ref


def krr_leg(torch, H, log, cg_iters=400, nrows=1024):
    """Kernel ridge regression at N = 2^22: points from a 32-component
    Gaussian mixture in [0,1]^3, Matern-3/2 with l = 0.1, (A + 1e-2 I) c = y,
    y = sin(2 pi p0) p1 + 0.01 xi; BF16 factors and near field with FP32
    arithmetic, the symmetric far field; ACA eps 1e-4, leaf 64, eta 1.5,
    k_max 64.  Build time, matvec time and bytes, the product's
    error on sampled rows against an FP64 dense product, and CG on the system
    (FP64 inner products) to relative residual 1e-6 or its breakdown."""
    n, ell, sigma2, eps = 1 << 22, 0.1, 1e-2, 1e-4
    pts = synth.gmm_points(n, 3, 31, dtype=np.float32)
    y = synth.krr_target(pts, 32, dtype=np.float32)
    pts_d = torch.from_numpy(pts).cuda()
    y_d = torch.from_numpy(y).cuda()
    kw = dict(compute_dtype="f32", storage_dtype="bf16", leaf_size=64, eta=1.5, aca_eps=eps,
              max_rank=64, sigma2=sigma2, symmetric_far=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hm = H.HMatrix(pts_d, "matern32", ell, **kw)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    st = hm.stats()
    log("bench: KRR 2^22 build %.2f s (phases %s), %d adm %d dense, factors %.3g entries, "
        "device %.1f GB" % (build_s, " ".join("%.0f" % v for v in st.phase_ms[:6]), st.n_adm,
                            st.n_dense, st.factor_entries, st.device_bytes / 1e9))
    stream = torch.cuda.current_stream()
    H.hmx_autotune(hm.h, 2, stream)
    x = torch.from_numpy(synth.normal_vector(n, 33, dtype=np.float32)).cuda()
    z = torch.empty_like(x)
    g = H.hmx_matvec_graph(hm.h, x, z)
    H.hmx_graph_launch(g, stream)
    H.hmx_profile_begin(hm.h, 5)
    for _ in range(5):
        H.hmx_matvec(hm.h, x, z, 1.0, 0.0, stream)
    phase_ms, calls = H.hmx_profile_end(hm.h)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    M = 10
    e0.record(stream)
    for _ in range(M):
        H.hmx_graph_launch(g, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    mv_ms = e0.elapsed_time(e1) / M
    H.hmx_graph_destroy(g)
    rows_d = torch.from_numpy(synth.sample_rows(n, nrows, 34)).cuda()
    ref = dense_rows_matern32(torch, pts_d, x, ell, rows_d) + sigma2 * x.double()[rows_d]
    err = (torch.linalg.norm(z.double()[rows_d] - ref) / torch.linalg.norm(ref)).item()
    # A's scale on the same rows: the product's error measured against the shift
    abs_err = (torch.linalg.norm(z.double()[rows_d] - ref) / torch.linalg.norm(
        x.double()[rows_d])).item()
    c = torch.zeros_like(y_d)
    t0 = time.perf_counter()
    s, it, res, tres = H.hmx_cg_solve(hm.h, y_d, c, rel_tol=1e-6, max_iter=cg_iters,
                                      raise_on_fail=False)
    cg_s = time.perf_counter() - t0
    msg = H.lib().hmx_last_error().decode() if s != H.HMX_OK else ""
    res_out = {
        "workload": "krr_gmm3d_n4m: N=2^22 points from a 32-component Gaussian mixture in "
                    "[0,1]^3 (seed 31), Matern-3/2 l=0.1, (A + 1e-2 I) c = y, y = sin(2 pi p0) "
                    "p1 + 0.01 xi; BF16 factors and near field, FP32 arithmetic, symmetric "
                    "far field; ACA eps 1e-4, leaf 64, eta 1.5, k_max 64",
        "build_s": build_s, "build_phase_ms": list(st.phase_ms), "n_adm": st.n_adm,
        "n_dense": st.n_dense, "sum_rank": st.sum_rank, "factor_entries": st.factor_entries,
        "near_entries": st.near_entries, "device_bytes": st.device_bytes,
        "matvec_ms": mv_ms, "matvec_phase_ms": list(phase_ms / max(calls, 1)),
        "matvec_bytes": st.matvec_bytes, "matvec_gbs": st.matvec_bytes / (mv_ms * 1e-3) / 1e9,
        "factor_bytes_read_per_matvec": (st.u_entries + st.v_entries) * st.entry_bytes,
        "factor_gbs": (st.u_entries + st.v_entries) * st.entry_bytes / (mv_ms * 1e-3) / 1e9,
        "near_evals_per_s": st.near_entries / (mv_ms * 1e-3),
        "rel_err_rows": err, "rows": nrows, "err_per_unit_x": abs_err,
        "cg": {"status": int(s), "iters": it, "rel_res": res, "true_rel_res": tres,
               "seconds": cg_s, "message": msg, "tol": 1e-6, "max_iter": cg_iters}}
    log("bench: KRR 2^22 matvec %.2f ms (%.3g B, %.0f GB/s), rel err %.2e on %d rows; CG status "
        "%d after %d iterations, res %.2e (%s)"
        % (mv_ms, st.matvec_bytes, res_out["matvec_gbs"], err, nrows, s, it, res, msg))
    hm.close()
    H.hmx_trim()
    return res_out


def krr_sizes_leg(torch, H, log, sizes=(1 << 14, 1 << 16, 1 << 18), max_iter=6000):
    """The kernel ridge regression system of the N = 2^22 configuration
    (32-component Gaussian mixture in [0,1]^3, Matern-3/2 l = 0.1,
    (A + 1e-2 I) c = y, CG to relative residual 1e-6, FP64 inner products) at
    sizes where the solve is affordable, in three arithmetics, each with the
    symmetric far field (H exactly symmetric), leaf 64, eta 1.5: FP64 (ACA eps
    1e-8), FP32 (eps 1e-6) and the configuration's own BF16 factors and near
    field (eps 1e-4).  Iterations, seconds, the recurrence and the true
    residual, or the breakdown (p.Ap <= 0: the operator is not definite)."""
    ell, sigma2 = 0.1, 1e-2
    forms = (("f64", dict(compute_dtype="f64", aca_eps=1e-8, max_rank=128)),
             ("f32", dict(compute_dtype="f32", aca_eps=1e-6, max_rank=96)),
             ("bf16", dict(compute_dtype="f32", storage_dtype="bf16", aca_eps=1e-4, max_rank=64)))
    out = {}
    for n in sizes:
        pts = synth.gmm_points(n, 3, 31)
        y = synth.krr_target(pts, 32)
        res_n = {}
        for form, kw in forms:
            dt = torch.float64 if form == "f64" else torch.float32
            pts_d = torch.from_numpy(pts).to(dt).cuda()
            y_d = torch.from_numpy(y).to(dt).cuda()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            hm = H.HMatrix(pts_d, "matern32", ell, leaf_size=64, eta=1.5, sigma2=sigma2,
                           symmetric_far=1, **kw)
            torch.cuda.synchronize()
            build_s = time.perf_counter() - t0
            H.hmx_autotune(hm.h, 2)
            c = torch.zeros_like(y_d)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, it, rres, tres = H.hmx_cg_solve(hm.h, y_d, c, rel_tol=1e-6, max_iter=max_iter,
                                                raise_on_fail=False)
            cg_s = time.perf_counter() - t0
            msg = H.lib().hmx_last_error().decode() if st != H.HMX_OK else ""
            res_n[form] = {"build_s": build_s, "status": int(st), "iters": it, "rel_res": rres,
                           "true_rel_res": tres, "cg_s": cg_s,
                           "ms_per_iter": 1e3 * cg_s / max(it, 1), "message": msg}
            log("bench: KRR N=%d %s: build %.2f s, CG status %d after %d iterations (%.2f s), "
                "res %.2e, true res %.2e %s" % (n, form, build_s, st, it, cg_s, rres, tres, msg))
            hm.close()
        out["n%d" % n] = res_n
    H.hmx_trim()
    return out


def batched_problems(torch, lo, hi, nprob=64):
    """nprob problems: N_p = round(2^U(lo, hi)), d_p in {2, 3}, points uniform,
    Gaussian p0 log-uniform in [0.005, 0.05] (seeds 41, 42, 4100 + p)."""
    g = synth.rng(41)
    ns = np.round(2.0 ** (lo + (hi - lo) * g.random(nprob))).astype(int)
    ds = g.integers(2, 4, nprob)
    p0s = synth.log_uniform(0.005, 0.05, nprob, 42)
    pts = [torch.from_numpy(synth.uniform_points(int(ns[q]), int(ds[q]), 4100 + q,
                                                 dtype=np.float32)).cuda() for q in range(nprob)]
    return ns, ds, p0s, pts


def multi_rhs_leg(torch, H, log, wl, pts_d, reps=5):
    """Several right-hand sides on the bench workload: m single-vector
    products against one hmx_matmat, for the plain FP32 and the BF16 forms
    (stored entries read once per 16 vectors instead of once per vector)."""
    n = wl["n"]
    out = {}
    for form, kw in (("plain_f32", dict(compute_dtype="f32")),
                     ("bf16", dict(compute_dtype="f32", storage_dtype="bf16")),
                     ("plain_f64", dict(compute_dtype="f64"))):
        hm = H.HMatrix(pts_d, wl["kernel"], wl["p0"], leaf_size=wl["leaf"], eta=wl["eta"],
                       aca_eps=wl["eps"], max_rank=wl["kmax"], **kw)
        st = hm.stats()
        dt = np.float64 if form == "plain_f64" else np.float32
        res = {}
        for m in (4, 16, 64):
            X = torch.from_numpy(synth.rng(7300 + m).standard_normal((m, n)).astype(dt)).cuda()
            Z = torch.empty_like(X)
            hm.matmat(X[:1], Z[:1])  # work vectors allocated outside the timing
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(reps):
                H.hmx_matmat(hm.h, X, Z)
            e1.record()
            torch.cuda.synchronize()
            mm_ms = e0.elapsed_time(e1) / reps
            z = torch.empty(n, dtype=X.dtype, device=X.device)
            e0.record()
            for _ in range(reps):
                for c in range(m):
                    H.hmx_matvec(hm.h, X[c], z)
            e1.record()
            torch.cuda.synchronize()
            mv_ms = e0.elapsed_time(e1) / reps
            ref = torch.empty(n, dtype=X.dtype, device=X.device)
            H.hmx_matvec(hm.h, X[m - 1], ref)
            err = (torch.linalg.norm(Z[m - 1].double() - ref.double()) /
                   torch.linalg.norm(ref.double())).item()
            res["m%d" % m] = {"matmat_ms": mm_ms, "matvecs_ms": mv_ms, "speedup": mv_ms / mm_ms,
                              "matrix_gbs_per_rhs": st.matvec_bytes * m / (mm_ms * 1e-3) / 1e9,
                              "rel_diff_last_column": err}
            log("bench: %s m=%d: matmat %.2f ms vs %d matvecs %.2f ms (%.2fx)"
                % (form, m, mm_ms, m, mv_ms, mv_ms / mm_ms))
        out[form] = res
        hm.close()
    return out


def batched_leg(torch, H, log, M=20):
    """64 independent problems as one block-diagonal handle against the same
    problems built (and multiplied) one by one, all on one stream.  The full
    recipe (N_p in [2^14, 2^18], 6.7M points) stores ~1e11 factor entries at
    eps 1e-5, beyond one GPU: it is built up to the ACA; build and matvec are
    compared on the same recipe with N_p in [2^12, 2^16]."""
    kw = dict(compute_dtype="f32", leaf_size=128, eta=1.5, aca_eps=1e-5, max_rank=64)
    stream = torch.cuda.current_stream()

    def timed(f):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = f()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    res = {}
    # the full recipe, up to the ACA
    ns, ds, p0s, pts = batched_problems(torch, 14, 18)
    H.HMatrix.batched(pts, "gaussian", list(p0s), aca_only=1, **kw).close()
    hb, tb = timed(lambda: H.HMatrix.batched(pts, "gaussian", list(p0s), aca_only=1, **kw))
    st = hb.stats()
    hb.close()
    t1 = 0.0
    for q in range(len(ns)):
        hq, t = timed(lambda: H.HMatrix(pts[q], "gaussian", float(p0s[q]), aca_only=1, **kw))
        t1 += t
        hq.close()
    res["aca_only"] = {"workload": "64 problems, N_p = round(2^U(14,18)) (total %d), d_p in "
                                   "{2,3}, Gaussian p0 log-uniform [0.005, 0.05], FP32, leaf 128, "
                                   "eta 1.5, eps 1e-5; build up to the ACA" % int(ns.sum()),
                       "batched_build_s": tb, "one_by_one_build_s": t1, "build_speedup": t1 / tb,
                       "n_adm": st.n_adm, "n_dense": st.n_dense, "aca_chunks": st.aca_chunks}
    log("bench: 64 problems (2^14-2^18, ACA only): batched build %.3f s, one by one %.3f s"
        % (tb, t1))
    del pts
    H.hmx_trim()
    # the reduced recipe, full builds and matvecs
    ns, ds, p0s, pts = batched_problems(torch, 12, 16)
    ntot = int(ns.sum())
    x = torch.from_numpy(synth.normal_vector(ntot, 4300, dtype=np.float32)).cuda()
    H.HMatrix.batched(pts, "gaussian", list(p0s), **kw).close()
    hb, tb = timed(lambda: H.HMatrix.batched(pts, "gaussian", list(p0s), **kw))
    st = hb.stats()
    H.hmx_autotune(hb.h, 3, stream)
    z = torch.empty_like(x)
    gr = H.hmx_matvec_graph(hb.h, x, z)
    H.hmx_graph_launch(gr, stream)
    _, tm = timed(lambda: [H.hmx_graph_launch(gr, stream) for _ in range(M)])
    H.hmx_graph_destroy(gr)
    hb.close()
    off = np.concatenate([[0], np.cumsum(ns)])
    t_build, t_mv = 0.0, 0.0
    for q in range(len(ns)):
        hq, t = timed(lambda: H.HMatrix(pts[q], "gaussian", float(p0s[q]), **kw))
        t_build += t
        xq = x[off[q]:off[q + 1]].contiguous()
        zq = torch.empty_like(xq)
        H.hmx_matvec(hq.h, xq, zq, 1.0, 0.0, stream)
        _, t = timed(lambda: [H.hmx_matvec(hq.h, xq, zq, 1.0, 0.0, stream) for _ in range(M)])
        t_mv += t
        hq.close()
    res["full"] = {"workload": "64 problems, N_p = round(2^U(12,16)) (total %d), d_p in {2,3}, "
                               "Gaussian p0 log-uniform [0.005, 0.05], FP32, leaf 128, eta 1.5, "
                               "eps 1e-5" % ntot,
                   "batched_build_s": tb, "batched_matvec_ms": tm / M * 1e3,
                   "batched_matvec_gbs": st.matvec_bytes / (tm / M) / 1e9,
                   "one_by_one_build_s": t_build, "one_by_one_matvec_ms": t_mv / M * 1e3,
                   "build_speedup": t_build / tb, "matvec_speedup": t_mv / tm,
                   "n_adm": st.n_adm, "n_dense": st.n_dense}
    log("bench: 64 problems (2^12-2^16): batched build %.3f s, matvec %.3f ms (%.0f GB/s); one "
        "by one build %.3f s, matvec %.3f ms" % (tb, tm / M * 1e3, res["full"]["batched_matvec_gbs"],
                                                  t_build, t_mv / M * 1e3))
    del pts
    H.hmx_trim()
    return res


def stream_copy_gbs(torch, dev, mib=4096, reps=5):
    """Bytes read + written per second of a plain device-to-device copy of
    mib MiB (torch's copy kernel), the best of reps: the box's measured
    stream bandwidth beside the HBM specification."""
    src = torch.ones(mib << 18, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del src, dst
    return 2.0 * (mib << 20) / (best * 1e-3) / 1e9


def cpu_baseline(wl, pts, x0, z_gpu_first, perm_gpu):
    """The oracle (FP64, stored mode) on a bounded sample of the workload: all
    leaves whose row cluster meets a contiguous range of Morton-order rows.
    Beside it, the measured FP64 form's product is checked against the
    oracle: against its H-matrix rows (same method, same arithmetic) and
    against its FP64 dense product on 4096 sampled rows (the tolerance
    10 eps + rounding)."""
    import oracle
    n = wl["n"]
    frac = wl.get("cpu_rows_frac", 1.0 / 32)
    nrows = max(wl["leaf"], int(n * frac))
    row_lo = (n - nrows) // 2
    row_hi = row_lo + nrows
    t0 = time.perf_counter()
    z_rows, perm, t = oracle.hmvp_rows(pts.astype(np.float64), x0.astype(np.float64),
                                       wl["kernel"], wl["p0"], wl["leaf"], wl["eta"], wl["kmax"],
                                       wl["eps"], row_lo, row_hi,
                                       eps0=1e-14)
    wall = time.perf_counter() - t0
    gbs = t["entries"] * 8 / t["apply_s"] / 1e9
    zg = z_gpu_first[perm[row_lo:row_hi]]
    err = float(np.linalg.norm(zg - z_rows) / np.linalg.norm(z_rows))
    assert np.array_equal(perm, perm_gpu), "GPU permutation differs from the oracle"
    rows = synth.sample_rows(n, 4096, 2201)
    zd = oracle.dense_matvec(pts.astype(np.float64), x0.astype(np.float64), wl["kernel"],
                             wl["p0"], rows=rows)
    err_dense = float(np.linalg.norm(z_gpu_first[rows] - zd) / np.linalg.norm(zd))
    return {
        "value": gbs, "unit": "GB/s", "cores": oracle.num_threads(), "kind": "oracle",
        "sample": "stored-mode H-matvec of Morton rows [%d, %d) (%d of %d rows, every leaf "
                  "meeting them built in FP64); apply %.3f s over %.3g stored entries" % (
                      row_lo, row_hi, nrows, n, t["apply_s"], t["entries"]),
        "build_s_sample": t["build_s"], "partition_s": t["partition_s"], "wall_s": wall,
        "gpu_f64_vs_oracle_hmatrix_rel_err": err,
        "gpu_f64_vs_oracle_dense_rel_err_4096rows": err_dense,
        "tolerance_10eps": 10 * wl["eps"],
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--matvecs", type=int, default=None)
    ap.add_argument("--workload", default="gauss2d_n1m_f32")
    ap.add_argument("--plain-eq-eps", type=float, default=None,
                    help="ACA eps of the equal-error plain form (default: searched)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-n22", action="store_true",
                    help="skip the N = 2^22 three-dimensional build comparison")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 64-problem batched build and matvec")
    ap.add_argument("--krr", action="store_true",
                    help="also run kernel ridge regression at N = 2^22 (Gaussian-mixture points, "
                         "Matern-3/2, BF16, CG): about a minute")
    ap.add_argument("--no-np", action="store_true",
                    help="skip the paper's N = 2^19 workload with and without precomputation")
    ap.add_argument("--np-large", action="store_true",
                    help="also the product without precomputation at N = 2^25 (d = 2, the "
                         "paper's largest) and N = 2^23 (d = 3): a few minutes")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the measured FP64 form (no predictor training, no other forms "
                         "or legs): the run the hardware counters are taken on")
    ap.add_argument("--leg", choices=("multi_rhs", "n22_aca", "n22_full", "aca_n20", "krr_sizes"),
                    default=None,
                    help="run one leg only and print its JSON (the runs the kernel-time and "
                         "counter summaries are taken on): several right-hand sides on the bench "
                         "workload, the N = 2^22 builds up to the ACA (with the one-shot learned "
                         "form), the N = 2^22 builds with the full learned/mixed and plain paths, "
                         "plain FP32 builds up to "
                         "the ACA on the bench workload, or the KRR system at N = 2^14 .. 2^18")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    import torch
    from paper_1708_09707_amd import hmx as H

    wl = dict(synth.WORKLOADS[args.workload])
    M = args.matvecs if args.matvecs is not None else wl.get("n_matvec", 10)
    n, d = wl["n"], wl["d"]
    dev = torch.device("cuda:0")
    log("bench: workload %s n=%d d=%d matvecs/step=%d steps=%d warmup=%d" % (
        args.workload, n, d, M, args.steps, args.warmup))
    copy_gbs = stream_copy_gbs(torch, dev)
    log("bench: device copy %.0f GB/s (read + write)" % copy_gbs)
    pts = synth.uniform_points(n, d, wl["pts_seed"], dtype=np.float32)
    nvec = min(M, 100)
    xs = [synth.normal_vector(n, wl["x_seed"] + k, dtype=np.float32) for k in range(nvec)]
    pts_d = torch.from_numpy(pts).to(dev)
    xs_d = [torch.from_numpy(x).to(dev) for x in xs]
    xs64_d = [x.double() for x in xs_d]  # the same values, for FP64 arithmetic
    rows_d = torch.from_numpy(synth.sample_rows(n, 256, 99)).to(dev)
    ref = dense_rows_fp64(torch, pts_d, xs_d[0], wl["p0"], rows_d)
    kern = H.make_kernel(wl["kernel"], wl["p0"])
    stream = torch.cuda.current_stream()

    if args.leg is not None:
        if args.leg == "multi_rhs":
            res = multi_rhs_leg(torch, H, log, wl, pts_d)
        elif args.leg == "n22_aca":
            res = n22_aca_builds(torch, H, log, full=False, one_shot=True)
        elif args.leg == "n22_full":
            res = n22_aca_builds(torch, H, log, full=True)
        elif args.leg == "krr_sizes":
            res = krr_sizes_leg(torch, H, log)
        else:
            res = {}
            for rep in range(3):
                hm = H.HMatrix(pts_d, wl["kernel"], wl["p0"], compute_dtype="f32",
                               leaf_size=wl["leaf"], eta=wl["eta"], aca_eps=wl["eps"],
                               max_rank=wl["kmax"], aca_only=1)
                st = hm.stats()
                res = {"aca_ms": st.phase_ms[3], "aca_kernel_evals": st.aca_kernel_evals,
                       "n_adm": st.n_adm, "sum_rank": st.sum_rank}
                log("bench: ACA-only build #%d: ACA %.1f ms" % (rep, st.phase_ms[3]))
                hm.close()
        print(json.dumps({"leg": args.leg, "workload": args.workload, args.leg: res}), flush=True)
        return
    mixed_eps = wl.get("mixed_eps", wl["eps"])
    mlp, train_info = (None, None) if args.headline_only else train_predictor(
        torch, H, wl, mixed_eps, log)

    def params(form, eps=None):
        o = dict(FORMS[form])
        if o.get("rank_mode") == "learned":
            o["mlp"] = mlp
        o.setdefault("compute_dtype", "f32")
        return H.hmx_params_default(leaf_size=wl["leaf"], eta=wl["eta"],
                                    aca_eps=wl["eps"] if eps is None else eps,
                                    max_rank=wl["kmax"], **o)

    def vectors(prm):
        return xs64_d if prm.compute_dtype == H.HMX_F64 else xs_d

    def one_step(prm, timed, label):
        xv = vectors(prm)
        z_d = torch.empty_like(xv[0])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = H.hmx_build(pts_d, kern, prm, stream)
        t1 = time.perf_counter()
        if tile_config[label] is None:
            # row-tile shape picked once per form by the library's autotuner
            tile_config[label], _ = H.hmx_autotune(h, 3, stream)
        else:
            H.hmx_set_tile_config(h, tile_config[label])
        H.hmx_profile_begin(h, M)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for k in range(M):
            H.hmx_matvec(h, xv[k % nvec], z_d, 1.0, 0.0, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        phase_ms, calls = H.hmx_profile_end(h)
        st = H.hmx_get_stats(h)
        rec = dict(build_s=t1 - t0, step_s=t2 - t0, mv_ms=e0.elapsed_time(e1) / M,
                   phase_ms=phase_ms / max(calls, 1), stats=st)
        if timed:
            log("bench: %s step build %.3f s, matvec %.3f ms (gather %.3f, phase1 %.3f, "
                "rowtile %.3f ms)" % (label, rec["build_s"], rec["mv_ms"], *rec["phase_ms"]))
        return h, rec

    tile_config = {}

    def run_form(prm, label, steps, warmup):
        tile_config.setdefault(label, None)
        for _ in range(warmup):
            h, _ = one_step(prm, False, label)
            H.hmx_destroy(h)
        recs = []
        for s in range(steps):
            h, rec = one_step(prm, True, label)
            if s < steps - 1:
                H.hmx_destroy(h)
            recs.append(rec)
        xv = vectors(prm)
        z0 = torch.empty_like(xv[0])
        H.hmx_matvec(h, xv[0], z0, 1.0, 0.0, stream)
        torch.cuda.synchronize()
        err = (torch.linalg.norm(z0.double()[rows_d] - ref) / torch.linalg.norm(ref)).item()
        st = recs[-1]["stats"]
        eager_ms = float(np.mean([r["mv_ms"] for r in recs]))
        # the matvec time: M replays of a captured one-matvec HIP graph
        zg = torch.empty_like(xv[0])
        g = H.hmx_matvec_graph(h, xv[0], zg)
        H.hmx_graph_launch(g, stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(M):
            H.hmx_graph_launch(g, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        mv_ms = e0.elapsed_time(e1) / M
        assert torch.equal(zg, z0), "graph replay differs from the eager matvec"
        H.hmx_graph_destroy(g)
        res = {
            "build_s": float(np.mean([r["build_s"] for r in recs])),
            "build_s_min": float(np.min([r["build_s"] for r in recs])),
            "matvec_ms": mv_ms,
            "matvec_eager_ms": eager_ms,
            "matvec_gbs": st.matvec_bytes / (mv_ms * 1e-3) / 1e9,
            "rel_err_256rows": err,
            "rowtile_ms": float(np.mean([r["phase_ms"][2] for r in recs])),
            "phase1_ms": float(np.mean([r["phase_ms"][1] for r in recs])),
            "build_phase_ms": list(st.phase_ms),
            "predict_ms": st.predict_ms,
            "aca_chunks": st.aca_chunks, "aca_capacity_entries": st.aca_capacity,
            "aca_fallback": st.aca_fallback, "aca_overflow": st.aca_overflow,
            "n_adm": st.n_adm, "n_dense": st.n_dense, "sum_rank": st.sum_rank,
            "max_rank": st.max_rank_used, "near_entries": st.near_entries,
            "factor_entries": st.factor_entries, "matvec_bytes": st.matvec_bytes,
            "device_bytes": st.device_bytes,
            "step_ms": 1e3 * float(np.mean([r["step_s"] for r in recs])),
            "rowtile_bytes": rowtile_bytes(st, xv[0].element_size()),
            "tile_config": tile_config[label],
            # the ACA (phase 3) and the tile-major pool phase (5, the near-field
            # evaluation and the factor rows) as work rates
            "aca_kernel_evals": st.aca_kernel_evals,
            "aca_evals_per_s": st.aca_kernel_evals / (st.phase_ms[3] * 1e-3),
            "aca_flops_per_s": st.aca_flops / (st.phase_ms[3] * 1e-3),
            "aca_flops_frac_fp32_peak": st.aca_flops / (st.phase_ms[3] * 1e-3) / FP32_PEAK,
            "near_evals_per_s": st.near_entries / (st.phase_ms[5] * 1e-3),
        }
        log("bench: %s build %.3f s, matvec %.3f ms (%.0f GB/s), rel err %.2e" % (
            label, res["build_s"], mv_ms, res["matvec_gbs"], err))
        return h, z0, res

    # the measured form (the printed value): the plain method in FP64, the
    # paper's arithmetic, on the workload's geometry, kernel and tolerance
    hD, zD, pd = run_form(params("plain_f64"), "plain_f64", args.steps, args.warmup)
    pd["aca_eps"] = wl["eps"]
    part_perm = H.hmx_get_partition(hD)["perm"]
    H.hmx_destroy(hD)
    z_f64_first = zD.cpu().numpy()
    H.hmx_trim()
    if args.headline_only:
        rt_gbs = pd["rowtile_bytes"] / (pd["rowtile_ms"] * 1e-3) / 1e9
        out = {"metric": METRIC, "value": pd["matvec_gbs"], "unit": "GB/s", "n_gpus": 1,
               "steps": args.steps, "warmup": args.warmup, "ms_per_step": pd["step_ms"],
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
               "dtype": "f64", "data": "synthetic", "plain_f64": pd,
               "roofline": {"kernel": "rowtile_kernel (FP64)", "bound": "hbm",
                            "achieved": rt_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": rt_gbs / HBM_PEAK_GBS,
                            "algorithmic_bytes_per_launch": pd["rowtile_bytes"],
                            "avg_launch_ms": pd["rowtile_ms"]}}
        if args.calibrate_copy > 0:
            nel = args.calibrate_copy * (1 << 20) // 4
            src = torch.ones(nel, dtype=torch.float32, device=dev)
            dst = torch.empty_like(src)
            torch.cuda.synchronize()
            dst.copy_(src)
            torch.cuda.synchronize()
            out["calibration_copy_bytes"] = nel * 4
        print(json.dumps(out), flush=True)
        return
    # the learned / mixed-precision form against the plain FP32 form (extra
    # keys; fewer steps)
    ext_steps = max(1, min(args.steps, 3))
    hL, zL, lm = run_form(params("learned_mixed", mixed_eps), "learned_mixed", ext_steps, 1)
    lm["aca_eps"] = mixed_eps
    H.hmx_destroy(hL)
    # the plain form at the workload's eps
    hP, zP, pl = run_form(params("plain"), "plain", ext_steps, 1)
    H.hmx_destroy(hP)
    # the plain form at equal error: the largest eps of the grid whose error
    # does not exceed learned_mixed's
    if args.plain_eq_eps is not None:
        eq_eps = args.plain_eq_eps
    else:
        eq_eps = wl["eps"]
        for e in EQ_GRID:
            h = H.hmx_build(pts_d, kern, params("plain", e), stream)
            z = torch.empty(n, dtype=torch.float32, device=dev)
            H.hmx_matvec(h, xs_d[0], z, 1.0, 0.0, stream)
            torch.cuda.synchronize()
            err = (torch.linalg.norm(z.double()[rows_d] - ref) / torch.linalg.norm(ref)).item()
            H.hmx_destroy(h)
            if err > lm["rel_err_256rows"]:
                break
            eq_eps = e
    hQ, _, pe = run_form(params("plain", eq_eps), "plain_eq(eps=%g)" % eq_eps, ext_steps, 1)
    H.hmx_destroy(hQ)
    pe["aca_eps"] = eq_eps

    rt_gbs = pd["rowtile_bytes"] / (pd["rowtile_ms"] * 1e-3) / 1e9
    traffic = measured_traffic(args.workload, "plain_f64", pd["tile_config"])
    out = {
        "metric": METRIC, "value": pd["matvec_gbs"], "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": pd["step_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "%s: N=%d points uniform in [0,1]^%d, %s kernel p0=%g, leaf %d, "
                               "eta %g, ACA eps %g, max rank %d; the plain method (adaptive "
                               "ACA, stored near field and factors) in FP64 arithmetic and "
                               "storage; %d matvecs per step" % (
                                   args.workload, n, d, wl["kernel"], wl["p0"], wl["leaf"],
                                   wl["eta"], wl["eps"], wl["kmax"], M),
                   "n": n, "d": d, "matvecs_per_step": M},
        "build_s": pd["build_s"], "matvec_ms": pd["matvec_ms"],
        "plain_f64": pd, "learned_mixed": lm, "plain": pl, "plain_equal_error": pe,
        "predictor_training": train_info,
        "vs_plain": {"build_speedup": pl["build_s"] / lm["build_s"],
                     "matvec_speedup": pl["matvec_ms"] / lm["matvec_ms"],
                     "build_speedup_equal_error": pe["build_s"] / lm["build_s"],
                     "matvec_speedup_equal_error": pe["matvec_ms"] / lm["matvec_ms"]},
        "matvec_roofline": {"bound": "hbm", "achieved": pd["matvec_gbs"], "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": pd["matvec_gbs"] / HBM_PEAK_GBS},
        "roofline": {"kernel": "rowtile_kernel (FP64)", "bound": "hbm", "achieved": rt_gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": rt_gbs / HBM_PEAK_GBS,
                     "traffic": traffic, "algorithmic_bytes_per_launch": pd["rowtile_bytes"],
                     "avg_launch_ms": pd["rowtile_ms"], "stream_copy_gbs": copy_gbs},
    }
    if args.calibrate_copy > 0:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters give
        # the scale between the counters and bytes moved
        nel = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = nel * 4
        del src, dst
    out["multi_rhs"] = multi_rhs_leg(torch, H, log, wl, pts_d)
    if not args.no_batched:
        H.hmx_trim()
        out["batched_64"] = batched_leg(torch, H, log)
    if not args.no_n22:
        # the N = 2^22 builds use nearly the whole device: return the library's
        # cached blocks and torch's reserve from the earlier legs to the driver
        H.hmx_trim()
        torch.cuda.empty_cache()
        out["n22_build"] = n22_aca_builds(torch, H, log)
    if args.krr:
        H.hmx_trim()
        out["krr_n4m"] = krr_leg(torch, H, log)
    paper_kw = dict(compute_dtype="f64", leaf_size=2048, eta=1.5, aca_eps=0.0, max_rank=16,
                    rank_mode="fixed")
    paper_desc = ("Halton points in [0,1]^2, unscaled Gaussian exp(-r^2), C_leaf 2048, eta 1.5, "
                  "fixed rank 16, FP64")
    if not args.no_np:
        out["paper_n512k"] = {
            "workload": "N=2^19 " + paper_desc,
            "paper_p100": {"setup_p_s": 1.3, "setup_np_s": 0.8, "matvec_p_s": 1.7,
                           "matvec_np_s": 2.7},
            **np_leg(torch, H, log, 1 << 19, 2, paper_kw)}
    if args.np_large:
        out["paper_n32m_np"] = {
            "workload": "N=2^25 " + paper_desc, "paper_p100": {"matvec_np_s": 360.0},
            **np_leg(torch, H, log, 1 << 25, 2, paper_kw, reps=1, forms=("np",))}
        out["gauss3d_n8m_np"] = {
            "workload": "N=2^23 uniform in [0,1]^3, gaussian p0=0.0145, leaf 64, eta 1.5, ACA eps "
                        "1e-5, max rank 64, FP32, symmetric far field, nothing stored",
            **np_leg(torch, H, log, 1 << 23, 3,
                     dict(compute_dtype="f32", leaf_size=64, eta=1.5, aca_eps=1e-5, max_rank=64,
                          symmetric_far=1),
                     p0=0.0145, reps=1, forms=("np",), points="uniform", seed=51)}
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle on a row sample)")
        out["cpu_baseline"] = cpu_baseline(wl, pts, xs[0], z_f64_first, part_perm)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
