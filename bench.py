#!/usr/bin/env python3
"""Throughput of the t-SVT ADMM step on one MI355X.

Workload: video-shaped tensor completion, 128 x 160 x 64 (a seeded smoothed
noise texture translated by (0.4, 0.7) px per frame, float32 values in
[0, 1]), 20% of the entries observed, fixed iteration count (tol = 0),
rho = 1e-2 grown by 1.1 per iteration up to 1e3.  One step = one ADMM
iteration: fused prologue + forward tube DFT, Jacobi SVD of the 33 Fourier
slices, shrink and rebuild, inverse DFT + fused dual update, control step.

`value` is the FP32 precision form (FP32 transforms, sweeps and rebuild;
FP64 rotation parameters, residual norms and stopping test): iterations/s
over --steps timed iterations (one tsvd_complete call of --steps iterations,
inputs resident in HBM, after a --warmup-iteration call).  The plain FP64
GPU path is timed the same way beside it, and the relative difference of
the two recovered tensors at the same iteration count is reported (the
FP64 path matches the FP64 oracle to ~1e-13, see the parity tests and the
`parity` field).  Also printed: the roofline of the dominant kernel of the
FP32 form, measured live with HIP events on the library's stream, and the
FP64 CPU oracle timed on a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "t-SVT ADMM iters/s vs FP64 plain at RSE≤1e-4; served p50/p99 solve latency"
SHAPE = (128, 160, 64)
PEAK_HBM_GBS = 8000.0          # MI355X HBM3E
PEAK_FP64_VALU_TFLOPS = 78.6   # MI355X FP64 vector
PEAK_FP32_VALU_TFLOPS = 157.3  # MI355X FP32 vector
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_video_completion.json")


def source_digest(files) -> str:
    """Digest of the sources a traffic record was measured with (the kernel's
    own file and the headers it includes): a record whose digest no longer
    matches describes an older kernel and is not reported."""
    h = hashlib.sha256()
    for rel in files:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(os.path.basename(rel).encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def roofline(stats: dict, steps: int, fp32: bool):
    """Dominant kernel family by summed event time, with achieved rate =
    algorithmic work / event time (both summed over its launches)."""
    name, st = max(stats.items(), key=lambda kv: kv[1]["total_ms"])
    secs = st["total_ms"] * 1e-3
    if st["work_is_bytes"]:
        achieved = st["work"] / secs / 1e9
        out = dict(bound="hbm", achieved=achieved, peak=PEAK_HBM_GBS, unit="GB/s")
    else:
        achieved = st["work"] / secs / 1e12
        peak = PEAK_FP32_VALU_TFLOPS if fp32 else PEAK_FP64_VALU_TFLOPS
        out = dict(bound="alu", achieved=achieved, peak=peak, unit="TFLOP/s")
    out["frac"] = out["achieved"] / out["peak"]
    out["kernel"] = name
    out["launches"] = st["launches"]
    out["avg_launch_us"] = st["total_ms"] * 1e3 / max(1, st["launches"])
    out["traffic"] = None
    try:
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("kernel") == name and tr.get("source_digest") == source_digest(tr["source_files"]):
            out["traffic"] = tr["bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        pass
    return out


def cpu_baseline(w, seconds: float):
    """The FP64 oracle on the same workload, timed for a bounded number of
    iterations (about `seconds` of CPU work)."""
    import numpy as np
    from oracle import admm

    try:
        from threadpoolctl import threadpool_info

        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    m_obs = np.asarray(w["M_obs"], dtype=np.float64)
    t0 = time.perf_counter()
    admm.complete(m_obs, w["mask"], w["rho"], w["growth"], w["rho_max"], max_iter=1, tol=0.0)
    one = time.perf_counter() - t0
    iters = int(max(1, min(200, seconds / max(one, 1e-3))))
    t0 = time.perf_counter()
    admm.complete(m_obs, w["mask"], w["rho"], w["growth"], w["rho_max"], max_iter=iters, tol=0.0)
    dt = time.perf_counter() - t0
    return dict(value=iters / dt, unit="iters/s", cores=threads, kind="oracle",
                sample=f"first {iters} ADMM iterations of the same 128x160x64 completion "
                       f"({dt:.1f} s, NumPy FP64, BLAS threads={threads})")


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--only", choices=["fp32", "fp64"], default=None,
                    help="run one form only (for profiler runs); prints its timing line")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain device copy of 1 GiB (reference for HBM byte counters) and exit")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(independent problems would shard with no communication).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1407_1785_amd as lib
    import workloads

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "device copy", "bytes_read": src.numel() * 8,
                          "bytes_written": dst.numel() * 8}), flush=True)
        return 0
    w = workloads.video_completion(0, shape=SHAPE)
    mask = torch.from_numpy(w["mask"]).to(dev)
    obs32 = torch.from_numpy(np.asarray(w["M_obs"], dtype=np.float32)).to(dev)
    obs64 = torch.from_numpy(np.asarray(w["M_obs"], dtype=np.float64)).to(dev)
    handle = lib.handle_for(obs32)
    kw = dict(rho=w["rho"], tol=0.0, growth=w["growth"], rho_max=w["rho_max"])
    fp32 = dict(precision=lib.PREC_FP32)

    if args.only:
        obs = obs32 if args.only == "fp32" else obs64
        extra = fp32 if args.only == "fp32" else {}
        if args.warmup > 0:
            lib.tsvd_complete(obs, mask, max_iter=args.warmup, **kw, **extra)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = lib.tsvd_complete(obs, mask, max_iter=args.steps, **kw, **extra)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        print(json.dumps({"form": args.only, "iters_per_s": args.steps / dt, "steps": args.steps,
                          "sweeps_per_iter": info.sweeps_total / max(1, info.iters)}), flush=True)
        return 0

    def timed(obs, **extra):
        if args.warmup > 0:
            lib.tsvd_complete(obs, mask, max_iter=args.warmup, **kw, **extra)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = lib.tsvd_complete(obs, mask, max_iter=args.steps, **kw, **extra)
        torch.cuda.synchronize()
        return x, info, time.perf_counter() - t0

    x32, info32, dt = timed(obs32, **fp32)
    x64, info64, dt64 = timed(obs64)
    value = args.steps / dt
    truth = np.asarray(w["X"], dtype=np.float64)
    x64n = x64.cpu().numpy()
    rse_forms = float(np.linalg.norm(x32.cpu().numpy().astype(np.float64) - x64n) / np.linalg.norm(x64n))

    result = {
        "metric": METRIC, "value": value, "unit": "iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "video-shaped TNN completion 128x160x64, 20% observed, "
                               "FP32 form (FP64 rotation parameters, norms and stop test), "
                               "fixed iterations",
                   "shape": list(SHAPE), "observed": 0.2, "precision": "fp32",
                   "iters_per_solve": args.steps},
        "fp64_plain": {"value": args.steps / dt64, "unit": "iters/s",
                       "ms_per_step": dt64 * 1e3 / args.steps,
                       "sweeps_per_iter": info64.sweeps_total / max(1, info64.iters)},
        "speedup_vs_fp64_plain": dt64 / dt,
        "rse_fp32_vs_fp64": rse_forms,
        "rse_bar": 1e-4,
        "sweeps_per_iter": info32.sweeps_total / max(1, info32.iters),
        "rse_vs_truth": float(np.linalg.norm(x64n - truth) / np.linalg.norm(truth)),
    }

    if not args.no_profile:
        handle.profile(True)
        lib.tsvd_complete(obs32, mask, max_iter=args.steps, **kw, **fp32)
        handle.profile(False)
        stats = handle.profile_read()
        result["roofline"] = roofline(stats, args.steps, fp32=True)
        result["kernels_ms_per_step"] = {k: v["total_ms"] / args.steps for k, v in stats.items()}

    # parity on a short prefix of the same solve (oracle vs GPU, FP64)
    from oracle import admm

    n_par = 3
    ref = admm.complete(np.asarray(w["M_obs"], dtype=np.float64), w["mask"], w["rho"],
                        w["growth"], w["rho_max"], max_iter=n_par, tol=0.0)
    den = np.linalg.norm(ref["X"])
    xp64, _ = lib.tsvd_complete(obs64, mask, max_iter=n_par, **kw)
    xp32, _ = lib.tsvd_complete(obs32, mask, max_iter=n_par, **kw, **fp32)
    result["parity"] = {"iters": n_par,
                        "fp64_rel_err_vs_oracle": float(np.linalg.norm(xp64.cpu().numpy() - ref["X"]) / den),
                        "fp32_rel_err_vs_oracle": float(np.linalg.norm(
                            xp32.cpu().numpy().astype(np.float64) - ref["X"]) / den)}

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
