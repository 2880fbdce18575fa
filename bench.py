"""Benchmark of the H-matrix hot path on one MI355X.

A step is one pass of the whole path over one synthetic point set: build
(ordering, cluster tree, block-tree traversal, batched ACA, near field,
matvec plan) followed by the workload's matvecs.  The line printed is

  value = H-matvec throughput in algorithmic GB/s (stored near field and
          factors read once, x / z / permutation once, t written and read),
plus build seconds, the roofline of the dominant kernel (the row-tile
matvec kernel, timed live with HIP events) and the CPU oracle timed on a
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "rowtile_traffic.json")


def kernel_source_hash() -> str:
    with open(os.path.join(ROOT, "paper_1708_09707_amd", "csrc", "k_mvp.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def rowtile_bytes(st) -> float:
    """Algorithmic bytes of one row-tile launch: the stored near field and U
    read once, t read once, z written once, the permutation read once.
    Re-reads of x|sigma segments served from cache are not counted."""
    esz = st.entry_bytes
    return (st.near_entries + st.u_entries) * esz + st.sum_rank * esz + st.n * (esz + 4)


def measured_traffic(workload: str):
    """HBM bytes per row-tile launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source") != kernel_source_hash() or rec.get("workload") != workload:
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(wl, pts, xs, z_gpu_first, perm_gpu):
    """The oracle (FP64, stored mode) on a bounded sample of the workload: all
    leaves whose row cluster meets a contiguous range of Morton-order rows."""
    import oracle
    n = wl["n"]
    frac = wl.get("cpu_rows_frac", 1.0 / 32)
    nrows = max(wl["leaf"], int(n * frac))
    row_lo = (n - nrows) // 2
    row_hi = row_lo + nrows
    t0 = time.perf_counter()
    z_rows, perm, t = oracle.hmvp_rows(pts.astype(np.float64), xs[0].astype(np.float64),
                                       wl["kernel"], wl["p0"], wl["leaf"], wl["eta"], wl["kmax"],
                                       wl["eps"], row_lo, row_hi,
                                       eps0=1e-7 if wl["dtype"] == "f32" else 1e-14)
    wall = time.perf_counter() - t0
    gbs = t["entries"] * 8 / t["apply_s"] / 1e9
    # the same rows of the GPU product (first matvec), Morton order
    zg = z_gpu_first[perm[row_lo:row_hi]]
    err = float(np.linalg.norm(zg - z_rows) / np.linalg.norm(z_rows))
    # brute-force FP64 rows as the exact reference
    rows = synth.sample_rows(n, 64, 99)
    zd = oracle.dense_matvec(pts.astype(np.float64), xs[0].astype(np.float64), wl["kernel"],
                             wl["p0"], rows=rows)
    err_dense = float(np.linalg.norm(z_gpu_first[rows] - zd) / np.linalg.norm(zd))
    assert np.array_equal(perm, perm_gpu), "GPU permutation differs from the oracle"
    return {
        "value": gbs, "unit": "GB/s", "cores": oracle.num_threads(), "kind": "oracle",
        "sample": "stored-mode H-matvec of Morton rows [%d, %d) (%d of %d rows, every leaf "
                  "meeting them built in FP64); apply %.3f s over %.3g stored entries" % (
                      row_lo, row_hi, nrows, n, t["apply_s"], t["entries"]),
        "build_s_sample": t["build_s"], "partition_s": t["partition_s"], "wall_s": wall,
        "gpu_vs_oracle_rel_err": err, "gpu_vs_dense_rel_err_64rows": err_dense,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--matvecs", type=int, default=None)
    ap.add_argument("--workload", default="gauss2d_n1m_f32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1708_09707_amd import hmx as H

    wl = dict(synth.WORKLOADS[args.workload])
    M = args.matvecs if args.matvecs is not None else wl.get("n_matvec", 10)
    n, d = wl["n"], wl["d"]
    npdt = np.float32 if wl["dtype"] == "f32" else np.float64
    tdt = torch.float32 if wl["dtype"] == "f32" else torch.float64
    dev = torch.device("cuda:0")
    print("bench: workload %s n=%d d=%d %s matvecs/step=%d steps=%d warmup=%d" % (
        args.workload, n, d, wl["dtype"], M, args.steps, args.warmup), file=sys.stderr,
        flush=True)
    pts = synth.uniform_points(n, d, wl["pts_seed"], dtype=npdt)
    nvec = min(M, 100)
    xs = [synth.normal_vector(n, wl["x_seed"] + k, dtype=npdt) for k in range(nvec)]
    pts_d = torch.from_numpy(pts).to(dev)
    xs_d = [torch.from_numpy(x).to(dev) for x in xs]
    z_d = torch.empty(n, dtype=tdt, device=dev)
    kern = H.make_kernel(wl["kernel"], wl["p0"])
    prm = H.hmx_params_default(leaf_size=wl["leaf"], eta=wl["eta"], aca_eps=wl["eps"],
                               max_rank=wl["kmax"], compute_dtype=wl["dtype"],
                               storage_dtype=wl.get("storage", wl["dtype"]))
    stream = torch.cuda.current_stream()

    def one_step(timed):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = H.hmx_build(pts_d, kern, prm, stream)
        t1 = time.perf_counter()
        H.hmx_profile_begin(h, M)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for k in range(M):
            H.hmx_matvec(h, xs_d[k % nvec], z_d, 1.0, 0.0, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        phase_ms, calls = H.hmx_profile_end(h)
        st = H.hmx_get_stats(h)
        rec = dict(build_s=t1 - t0, step_s=t2 - t0, mv_ms=e0.elapsed_time(e1) / M,
                   phase_ms=phase_ms / max(calls, 1), stats=st)
        if timed:
            print("bench: step build %.3f s, matvec %.3f ms (gather %.3f, phase1 %.3f, "
                  "rowtile %.3f ms)" % (rec["build_s"], rec["mv_ms"], *rec["phase_ms"]),
                  file=sys.stderr, flush=True)
        return h, rec

    for _ in range(args.warmup):
        h, _ = one_step(False)
        H.hmx_destroy(h)
    recs = []
    torch.cuda.synchronize()
    for s in range(args.steps):
        h, rec = one_step(True)
        if s < args.steps - 1:
            H.hmx_destroy(h)
        recs.append(rec)
    torch.cuda.synchronize()
    # keep the last handle for the checks below
    st = recs[-1]["stats"]
    z_first = torch.empty(n, dtype=tdt, device=dev)
    H.hmx_matvec(h, xs_d[0], z_first, 1.0, 0.0, stream)
    torch.cuda.synchronize()
    part_perm = H.hmx_get_partition(h)["perm"]
    H.hmx_destroy(h)
    z_first = z_first.double().cpu().numpy()

    mv_ms = float(np.mean([r["mv_ms"] for r in recs]))
    build_s = float(np.mean([r["build_s"] for r in recs]))
    step_ms = 1e3 * float(np.mean([r["step_s"] for r in recs]))
    rt_ms = float(np.mean([r["phase_ms"][2] for r in recs]))
    gbs = st.matvec_bytes / (mv_ms * 1e-3) / 1e9
    rt_bytes = rowtile_bytes(st)
    rt_gbs = rt_bytes / (rt_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.workload)
    out = {
        "metric": METRIC, "value": gbs, "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": step_ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": wl.get("storage", wl["dtype"]),
        "data": "synthetic",
        "config": {"workload": "%s: plain method, N=%d points uniform in [0,1]^%d, %s kernel "
                               "p0=%g, leaf %d, eta %g, ACA eps %g, max rank %d, %s arithmetic, "
                               "%s storage, %d matvecs per step" % (
                                   args.workload, n, d, wl["kernel"], wl["p0"], wl["leaf"],
                                   wl["eta"], wl["eps"], wl["kmax"], wl["dtype"],
                                   wl.get("storage", wl["dtype"]), M),
                   "n": n, "d": d, "matvecs_per_step": M},
        "build_s": build_s, "matvec_ms": mv_ms,
        "build_phase_ms": list(recs[-1]["stats"].phase_ms),
        "partition": {"n_adm": st.n_adm, "n_dense": st.n_dense, "levels": st.levels,
                      "sum_rank": st.sum_rank, "max_rank": st.max_rank_used,
                      "near_entries": st.near_entries, "factor_entries": st.factor_entries,
                      "matvec_bytes": st.matvec_bytes, "device_bytes": st.device_bytes},
        "matvec_roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": gbs / HBM_PEAK_GBS},
        "roofline": {"kernel": "rowtile_kernel", "bound": "hbm", "achieved": rt_gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": rt_gbs / HBM_PEAK_GBS,
                     "traffic": traffic, "algorithmic_bytes_per_launch": rt_bytes,
                     "avg_launch_ms": rt_ms},
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
    if not args.no_cpu_baseline:
        print("bench: cpu baseline (oracle on a row sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, pts, xs, z_first, part_perm)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
