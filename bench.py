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
the two recovered tensors at the same iteration count is reported.  The
`parity` field compares both timed outputs with the FP64 oracle run for
the same --steps iterations (whole tensor, largest Fourier slice, largest
tube), and `cpu_baseline` is that oracle run's rate on the host's threads,
with a short single-thread sample beside it.  Also printed: the roofline of
the dominant kernel of each form (n(n-1)/2 (28m+20n) flops per slice sweep
from the device's per-slice sweep sums, HIP events on the library's
stream, HBM traffic from the committed counter record while its source
digest matches), the DFT passes' HBM fraction and the rebuild's matrix-core
fraction at the kept rank, and the batched, serving, full-size RPCA,
compression, sampling-sweep and tube-RPCA legs.  `--gpus N` with N > 1
exits with a message: the library runs on one GPU.
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
PEAK_FP32_MATRIX_TFLOPS = 157.3  # MI355X FP32 matrix cores (dense)
PEAK_FP64_MATRIX_TFLOPS = 78.6   # MI355X FP64 matrix cores (dense)
# Stopping tolerance of the FP32 form where a workload asks for less: a
# relative residual of 1e-7 is below one FP32 unit (1.19e-7), so the FP32
# iterates cannot meet it and only drift once the penalty is large.
FP32_TOL_FLOOR = 1e-6
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


def roofline(stats: dict, fp32: bool, m: int, n: int):
    """Dominant kernel family by summed event time (HIP events on the
    library's stream), with achieved rate = algorithmic work / event time.

    For the Jacobi families the work is n (n - 1) / 2 (28 m + 20 n) flops
    per slice sweep (one complex dot product over the m slice rows and two
    rotated columns of m + n stacked rows per visited pair), from the summed
    per-slice sweep counts the library records; the figure that counts only
    what was applied (16 m per visited pair, 16 (m + n) per applied rotation)
    is given beside it.  Peaks: FP32 vector 157.3 TFLOP/s (packed two-wide
    FMAs), 78.6 without packing (what these kernels are compiled to), FP64 78.6."""
    name, st = max(stats.items(), key=lambda kv: kv[1]["total_ms"])
    secs = st["total_ms"] * 1e-3
    launches = max(1, st["launches"])
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
    out["avg_launch_us"] = st["total_ms"] * 1e3 / launches
    out["work_per_launch"] = st["work"] / launches
    if st.get("slice_sweeps"):
        applied = 16.0 * m * st["pairs_visited"] + 16.0 * (m + n) * st["rotations"]
        out["model"] = "n(n-1)/2 (28m+20n) flops per slice sweep"
        out["slice_sweeps_per_launch"] = st["slice_sweeps"] / launches
        out["rotations_per_launch"] = st["rotations"] / launches
        out["pairs_per_launch"] = st["pairs_visited"] / launches
        out["frac_of_78.6_nonpacked"] = out["achieved"] / PEAK_FP64_VALU_TFLOPS
        out["achieved_applied_only"] = applied / secs / 1e12
    out["traffic"] = None
    try:
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        form = "fp32" if fp32 else "fp64"
        if (tr.get("kernel") == name and tr.get("precision") == form
                and tr.get("source_digest") == source_digest(tr["source_files"])):
            out["traffic"] = tr["bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        pass
    return out


def device_copy_gbs(torch, nbytes: int = 1 << 30, reps: int = 5) -> float:
    """Read + write rate of a plain device-to-device copy of `nbytes` (the
    best of `reps`, HIP events on torch's stream): the practical ceiling the
    HBM-bound passes are also compared with."""
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b) * 1e-3)
    del src, dst
    return 2.0 * nbytes / best / 1e9


def side_rooflines(stats: dict, fp32: bool, m: int, n: int, h: int, copy_gbs: float = 0.0):
    """The HBM fraction of the two DFT passes (with the fused prologue and
    epilogue; algorithmic bytes per launch) and the matrix-core fraction of
    the rebuild W diag(d) V^H, counted at the kept rank (8 m n r_k flops per
    slice, the useful product) and dense (8 m n^2, what it computes), and,
    since at these ranks it is memory-bound, its bytes (W, V read, Zhat
    written, h slices) against the HBM peak.  The DFT passes are also given
    against `copy_gbs`, the rate of a plain device copy measured here."""
    out = {}
    for fam in ("dft_forward", "dft_inverse"):
        st = stats.get(fam)
        if st and st["total_ms"] > 0:
            gbs = st["work"] / (st["total_ms"] * 1e-3) / 1e9
            out[fam] = {"achieved_GBs": gbs, "peak_GBs": PEAK_HBM_GBS, "frac": gbs / PEAK_HBM_GBS,
                        "avg_launch_us": st["total_ms"] * 1e3 / max(1, st["launches"]),
                        "bytes_per_launch": st["work"] / max(1, st["launches"])}
            if copy_gbs > 0:
                out[fam]["copy_GBs"] = copy_gbs
                out[fam]["frac_of_copy"] = gbs / copy_gbs
    st = stats.get("svt_rebuild")
    if st and st["total_ms"] > 0:
        secs = st["total_ms"] * 1e-3
        peak = PEAK_FP32_MATRIX_TFLOPS if fp32 else PEAK_FP64_MATRIX_TFLOPS
        kept_flops = 8.0 * m * n * st["kept_rank"]
        out["svt_rebuild"] = {"bound": "mfma", "peak_TFs": peak,
                              "kept_rank_per_launch": st["kept_rank"] / max(1, st["launches"]),
                              "achieved_TFs_kept_rank": kept_flops / secs / 1e12,
                              "frac_kept_rank": kept_flops / secs / 1e12 / peak,
                              "achieved_TFs_dense": st["work"] / secs / 1e12,
                              "frac_dense": st["work"] / secs / 1e12 / peak,
                              "avg_launch_us": st["total_ms"] * 1e3 / max(1, st["launches"])}
        # at these ranks the product is memory-bound: W (m x n) and V (n x n)
        # read, Zhat (m x n) written, complex, per slice
        b = 4 if fp32 else 8
        byt = st["launches"] * h * (2.0 * m * n + n * n) * 2 * b
        out["svt_rebuild"]["bytes_per_launch"] = byt / max(1, st["launches"])
        out["svt_rebuild"]["achieved_GBs"] = byt / secs / 1e9
        out["svt_rebuild"]["frac_hbm"] = byt / secs / 1e9 / PEAK_HBM_GBS
    return out


def batched_leg(lib, torch, np, workloads, iters: int):
    """64 uneven completion problems (n1, n2 ~ U{48..320}, n3 ~ U{8..128},
    tubal rank ~ U{2..10}, Bernoulli(p ~ U[0.2, 0.6]) masks), FP32 form, a
    fixed number of iterations each, solved together by tsvd_batch_run.
    A short run over the same problems first lets the block-width tuner see
    every shape class (its choices are cached for the process).  Returns the
    leg's figures and its smallest problem (inputs and GPU result) for the
    oracle comparison of the CPU leg."""
    specs = workloads.batch_specs(0)
    probs, data = [], []
    for i, sp in enumerate(specs):
        b = workloads.batch_problem(sp, i, iters=iters)
        y = torch.from_numpy(b["M_obs"].astype(np.float32)).cuda()
        m = torch.from_numpy(b["mask"]).cuda()
        probs.append(lib.complete_problem(y, m, rho=b["rho"], tol=0.0, growth=b["growth"],
                                          rho_max=b["rho_max"], max_iter=iters))
        data.append(b)
    print("[bench] batched leg: problems staged, tuning run", file=sys.stderr, flush=True)
    lib.batch_run([lib.complete_problem(p.x, p.mask, 1e-2, 0.0, max_iter=2) for p in probs])
    torch.cuda.synchronize()
    print("[bench] batched leg: timed run", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    res = lib.batch_run(probs)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    elems = sum(int(np.prod(d["M_obs"].shape)) for d in data)
    slices = sum(sp["n3"] // 2 + 1 for sp in specs)
    out = {"workload": "64 uneven completion problems, n1,n2~U{48..320}, n3~U{8..128}, rank~U{2..10}, "
                       "p~U[0.2,0.6], FP32 form", "problems": len(probs), "iters_per_solve": iters,
           "elements": elems, "slices": slices, "seconds": dt, "solves_per_s": len(probs) / dt,
           "iters_per_s": len(probs) * iters / dt,
           "statuses_ok": all(st == 0 for st, _ in res),
           "sweeps_per_iter_mean": float(np.mean([i.sweeps_total / max(1, i.iters) for _, i in res]))}
    # the observed entries are kept exactly; the smallest problem goes to the
    # CPU leg for the oracle comparison at the same iteration count
    out["observed_kept_exactly"] = all(
        bool(np.array_equal(p.out.cpu().numpy()[d["mask"].astype(bool)],
                            d["M_obs"].astype(np.float32)[d["mask"].astype(bool)])) for p, d in zip(probs, data))
    k = int(np.argmin([d["M_obs"].size for d in data]))
    out["sampled_shape"] = list(data[k]["M_obs"].shape)
    case = {"data": data[k], "iters": iters, "got": probs[k].out.cpu().numpy().astype(np.float64)}
    return out, case


def compression_leg(lib, torch, np, workloads):
    """Sec. 3 on the synthetic video (the completion workload's full
    128 x 160 x 64 tensor): the explicit t-SVD factors (FP64 path and FP32
    form) and Methods 1 and 2 at compression ratios near 5, 10, 20 and 40,
    each timed on the GPU as the mean of 3 calls after one untimed call, with
    RSE in dB (20 log10 of the relative Frobenius error, as Sec. 3 plots it).
    Returns the figures and one Method 1 result for the CPU leg's oracle
    comparison."""
    x = np.asarray(workloads.video_completion(0, shape=SHAPE)["X"], dtype=np.float64)
    n1, n2, n3 = x.shape
    xg = torch.from_numpy(x).cuda()
    xg32 = xg.float()

    def timed(fn, reps=3):
        r = fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        return r, (time.perf_counter() - t0) / reps

    def rse_db(a):
        a = a.cpu().numpy().astype(np.float64)
        return float(20.0 * np.log10(np.linalg.norm(a - x) / np.linalg.norm(x)))

    _, t64 = timed(lambda: lib.tsvd_factors(xg))
    _, t32 = timed(lambda: lib.tsvd_factors(xg32, precision=lib.PREC_FP32))
    curve = []
    for target in (5, 10, 20, 40):
        k2 = max(1, round(n1 * n2 * n3 / (target * (n1 + n2 + 1))))
        k3 = max(1, round(n1 * n2 / (target * (n1 + n2 + 1))))
        (m1, r1), t1 = timed(lambda: lib.compress(xg, lib.COMPRESS_TSVD, k2))
        (m2, r2), t2 = timed(lambda: lib.compress(xg, lib.COMPRESS_TUBAL, k3))
        curve.append({"target_ratio": target,
                      "method1": {"k2": k2, "ratio": r1, "rse_db": rse_db(m1), "ms": t1 * 1e3},
                      "method2": {"k3": k3, "ratio": r2, "rse_db": rse_db(m2), "ms": t2 * 1e3}})
    k2 = curve[1]["method1"]["k2"]
    got = lib.compress(xg, lib.COMPRESS_TSVD, k2)[0].cpu().numpy()
    out = {"workload": "t-SVD factors and compression (Sec. 3) of the synthetic 128x160x64 video",
           "factors_ms_fp64": t64 * 1e3, "factors_ms_fp32": t32 * 1e3, "curve": curve}
    return out, {"x": x, "k2": k2, "got": got}


def sweep_leg(lib, torch, np, workloads, iters: int):
    """Sampling-rate sweep (the Sec. 6 completion experiment on synthetic
    videos): RSE in dB of TNN completion (this solver on the tensor) and of
    the vectorised matrix nuclear-norm baseline (the same solver with n3 = 1
    on the n1 n2 x n3 unfolding, the frontal slices as columns), rates
    10%..90%, 3-D video 128x160x64 and 4-D colour video 96x128x3x48, FP32
    form, at most `iters` iterations with tol 1e-6.  Returns the figures and a
    short FP64 prefix of the 3-D baseline at 50% for the CPU leg's oracle
    comparison."""
    sw = workloads.sampling_sweep(0)
    kw = dict(rho=sw["rho"], growth=sw["growth"], rho_max=sw["rho_max"], tol=1e-6, max_iter=iters,
              precision=lib.PREC_FP32)

    def solve(x, mask, shape):
        xs = torch.from_numpy(np.ascontiguousarray((x * mask).reshape(shape))).float().cuda()
        ms = torch.from_numpy(np.ascontiguousarray(mask.reshape(shape))).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out, info = lib.tsvd_complete(xs, ms, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        o = out.cpu().numpy().astype(np.float64).reshape(x.shape)
        rse = np.linalg.norm(o - x) / np.linalg.norm(x)
        return {"rse_db": float(20.0 * np.log10(rse)), "iters": int(info.iters), "seconds": dt}

    rows = []
    for p, (m3, m4) in sw["masks"].items():
        v3, v4 = sw["video3"].astype(np.float64), sw["video4"].astype(np.float64)
        rows.append({"rate": p,
                     "video3_tnn": solve(v3, m3, v3.shape),
                     "video3_matrix": solve(v3, m3, (128 * 160, 64, 1)),
                     "video4_tnn": solve(v4, m4, v4.shape),
                     "video4_matrix": solve(v4, m4, (96 * 128, 3 * 48, 1))})
    print(f"[bench] sweep leg: {len(rows)} rates", file=sys.stderr, flush=True)
    # FP64 prefix of the 3-D baseline at 50% for the oracle comparison
    m3 = sw["masks"][0.5][0]
    y = (sw["video3"].astype(np.float64) * m3).reshape(128 * 160, 64, 1)
    mk = m3.reshape(128 * 160, 64, 1)
    got, _ = lib.tsvd_complete(torch.from_numpy(y).cuda(), torch.from_numpy(mk).cuda(), rho=sw["rho"],
                               growth=sw["growth"], rho_max=sw["rho_max"], tol=0.0, max_iter=5)
    out = {"workload": "sampling sweep 10-90%: TNN vs vectorised matrix nuclear norm, synthetic 3-D and 4-D "
                       "videos, FP32 form", "max_iter": iters, "rows": rows}
    case = {"y": y, "mask": mk, "iters": 5, "rho": sw["rho"], "growth": sw["growth"], "rho_max": sw["rho_max"],
            "got": got.cpu().numpy()}
    return out, case


def tube_rpca_leg(lib, torch, np, workloads):
    """The Sec. 5 RPCA experiment on a synthetic 72x128x80 video with
    tube-block noise (the same pixels within each 10-frame block): tensor
    RPCA with the tube shrink (lam = 1/sqrt(max(n1, n2))) against matrix RPCA
    on the n1 n2 x n3 unfolding (entrywise shrink, lam = 1/sqrt(max(n1 n2,
    n3))), both through this solver in the FP32 form.  Reported: RSE of L in
    dB against the clean video, F1 of the recovered noise support (|S| >
    1e-3 max|M|) and time.  Returns the figures and FP64 25-iteration
    prefixes of both for the CPU leg's oracle comparison."""
    w = workloads.tube_block_video(0)
    m = w["M"]
    n1, n2, n3 = m.shape
    kw = dict(mu=w["mu"], tol=w["tol"], growth=w["growth"], mu_max=w["mu_max"], max_iter=w["max_iter"])

    def run(shape, lam, shrink, prec=lib.PREC_FP32, **extra):
        x = torch.from_numpy(np.ascontiguousarray(m.reshape(shape)))
        x = (x.float() if prec == lib.PREC_FP32 else x).cuda()
        args = dict(kw, **extra)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lo, sp, info = lib.trpca(x, lam, shrink=shrink, precision=prec, **args)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return lo.cpu().numpy().astype(np.float64).reshape(m.shape), sp.cpu().numpy().astype(np.float64).reshape(
            m.shape), info, dt

    def figures(lo, sp, info, dt):
        pred = np.abs(sp) > 1e-3 * np.abs(m).max()
        truth = w["S"] != 0
        tp = np.count_nonzero(pred & truth)
        f1 = 2.0 * tp / max(1, 2 * tp + np.count_nonzero(pred & ~truth) + np.count_nonzero(~pred & truth))
        rse = np.linalg.norm(lo - w["L"]) / np.linalg.norm(w["L"])
        return {"rse_l_db": float(20.0 * np.log10(rse)), "support_f1": float(f1), "iters": int(info.iters),
                "converged": bool(info.converged), "seconds": dt}

    tensor = figures(*run(m.shape, w["lam_tensor"], lib.SHRINK_L112))
    matrix = figures(*run((n1 * n2, n3, 1), w["lam_matrix"], lib.SHRINK_L1))
    # 25 iterations: the penalty has grown enough for S to be non-zero (lam/mu starts near 90)
    pre_t = run(m.shape, w["lam_tensor"], lib.SHRINK_L112, lib.PREC_FP64, max_iter=25, tol=0.0)
    pre_m = run((n1 * n2, n3, 1), w["lam_matrix"], lib.SHRINK_L1, lib.PREC_FP64, max_iter=25, tol=0.0)
    out = {"workload": "tube-block noise on a synthetic 72x128x80 video: tensor RPCA (tube shrink) vs matrix RPCA "
                       "on the unfolding, FP32 form", "noise": "2% of pixels per 10-frame block, N(0, 0.25)",
           "tensor_rpca": tensor, "matrix_rpca": matrix}
    case = {"m": m, "lam_tensor": w["lam_tensor"], "lam_matrix": w["lam_matrix"], "mu": w["mu"],
            "growth": w["growth"], "mu_max": w["mu_max"], "iters": 25,
            "got_tensor": (pre_t[0], pre_t[1]), "got_matrix": (pre_m[0], pre_m[1])}
    return out, case


def trpca_256_leg(lib, torch, np, workloads):
    """The tensor-RPCA workload of Sec. 5 at full size (256 x 256 x 64,
    tubal rank 5, 10% entrywise corruption U[-1, 1], lambda = 1/128, mu0 =
    1e-3 grown by 1.2, tol 1e-7, entrywise l1), solved to its stopping rule
    in the FP32 form and on the plain FP64 path: iterations, time,
    iterations/s, RSE of L against the planted part, support F1 of S, and the
    FP32 form's L against the FP64 path's."""
    from oracle import metrics

    p = workloads.trpca_problem(0)
    res = {}
    outs = {}
    for form, dt, prec in (("fp32", torch.float32, lib.PREC_FP32), ("fp64", torch.float64, lib.PREC_FP64)):
        x = torch.from_numpy(p["M"]).to(dt).cuda()
        # the FP32 form stops at 1e-6: the workload's 1e-7 is below one FP32 unit of relative change
        tol = max(p["tol"], FP32_TOL_FLOOR) if form == "fp32" else p["tol"]
        lib.trpca(x, p["lam"], p["mu"], 0.0, growth=p["growth"], mu_max=p["mu_max"], max_iter=2, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lo, sp, info = lib.trpca(x, p["lam"], p["mu"], tol, growth=p["growth"], mu_max=p["mu_max"],
                                 max_iter=p["max_iter"], precision=prec)
        torch.cuda.synchronize()
        dt_s = time.perf_counter() - t0
        lo = lo.cpu().numpy().astype(np.float64)
        sp = sp.cpu().numpy().astype(np.float64)
        outs[form] = lo
        res[form] = {"tol": tol, "iters": int(info.iters), "converged": bool(info.converged), "seconds": dt_s,
                     "iters_per_s": info.iters / dt_s, "primal": info.primal, "change": info.change,
                     "sweeps_per_iter": info.sweeps_total / max(1, info.iters),
                     "rse_l": metrics.rse(lo, p["L"]), "rse_l_db": metrics.rse_db(lo, p["L"]),
                     "support_f1": metrics.support_f1(sp, p["S"], p["M"])}
    res["workload"] = ("tensor RPCA 256x256x64, rank 5, 10% entrywise corruption, lambda=1/128, mu0=1e-3 x1.2, "
                       "l1 shrink, to the stopping rule: tol 1e-7 (FP64), 1e-6 (FP32 form)")
    res["fp32_l_rel_diff_vs_fp64"] = float(np.linalg.norm(outs["fp32"] - outs["fp64"]) /
                                           np.linalg.norm(outs["fp64"]))
    return res


def serving_leg(lib, torch, np, workloads, rate: float, window: float, budget_gb: float, limit_s: float = 240.0):
    """The serving mix: Poisson arrivals at `rate` per second during `window`
    seconds (70% completion / 30% tensor RPCA, 10% 4-D colour video, other
    shapes as in the batched workload; FP32 form; at most 150 iterations,
    tol 1e-7).  Every request is submitted at its arrival time to the
    handle's serving worker; latency = completion - arrival.  After
    `limit_s` seconds the requests still open are cancelled and counted as
    unfinished."""
    reqs = workloads.arrivals(0, rate, window)
    staged = []
    for r in reqs:
        d = workloads.serve_request(r)
        if d["kind"] == "complete":
            y = torch.from_numpy(d["M_obs"].astype(np.float32)).cuda()
            m = torch.from_numpy(d["mask"]).cuda()
            p = lib.complete_problem(y, m, d["rho"], max(d["tol"], FP32_TOL_FLOOR), d["growth"], d["rho_max"],
                                     d["max_iter"])
        else:
            x = torch.from_numpy(d["M"].astype(np.float32)).cuda()
            p = lib.trpca_problem(x, d["lam"], d["mu"], max(d["tol"], FP32_TOL_FLOOR), lib.SHRINK_L1, d["growth"],
                                  d["mu_max"], d["max_iter"])
        staged.append((r["t"], p))
    torch.cuda.synchronize()
    print(f"[bench] serving leg: {len(staged)} requests staged", file=sys.stderr, flush=True)
    handle = lib.Handle(0, hbm_budget_bytes=int(budget_gb * (1 << 30)))
    pending, lat, iters, statuses = {}, [], [], []
    t0 = time.perf_counter()
    nxt = 0
    last_done = t0
    unfinished = 0
    try:
        while nxt < len(staged) or pending:
            now = time.perf_counter() - t0
            if now > limit_s:
                for t in list(pending):
                    lib.cancel(t, handle)
                unfinished = len(pending) + len(staged) - nxt
                print(f"[bench] serving leg: wall-clock limit, {unfinished} requests unfinished",
                      file=sys.stderr, flush=True)
                break
            while nxt < len(staged) and staged[nxt][0] <= now:
                pending[lib.submit(staged[nxt][1], handle)] = staged[nxt][0]
                nxt += 1
            for t in list(pending):
                r = lib.poll(t, handle)
                if r is not None:
                    st, info = r
                    lat.append(info.seconds)
                    iters.append(info.iters)
                    statuses.append(st)
                    del pending[t]
                    last_done = time.perf_counter()
                    if len(lat) % 20 == 0:
                        print(f"[bench] serving leg: {len(lat)} done", file=sys.stderr, flush=True)
            time.sleep(0.0005)
        stats = lib.serve_stats(handle)
    finally:
        handle.close()
    span = last_done - t0
    lat = np.asarray(lat)
    return {"workload": f"Poisson {rate:g} req/s for {window:g} s: 70% completion / 30% TRPCA, 10% 4-D "
                        "96x128x3x48 colour video, else shapes as the batched workload; FP32 form, "
                        "<=150 iterations, tol 1e-6 (the FP32 form's floor; the mix asks 1e-7)",
            "requests": len(staged), "unfinished": unfinished, "solves_per_s": len(lat) / span, "span_s": span,
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "max_s": float(lat.max()), "mean_iters": float(np.mean(iters)),
            "statuses_ok": all(s == 0 for s in statuses), "peak_running": stats["peak_running"],
            "arena_gb": stats["arena_bytes"] / (1 << 30)}


def cpu_baseline(w, cases: dict, single_iters: int):
    """The FP64 oracle on the host.  Timed: the same completion as the timed
    GPU steps, for as many iterations (all host cores: NumPy with its BLAS
    threads), and its first `single_iters` iterations with one BLAS thread.
    The first run is also the reference of the parity check at the timed
    iteration count.  Also the reference results of the GPU legs'
    comparison cases (not timed, except the t-SVD of the compression leg).
    Returns (baseline, comparisons)."""
    import numpy as np
    from oracle import admm
    from oracle import compress as ocompress
    from oracle import tensor as otensor
    from threadpoolctl import threadpool_info, threadpool_limits

    from tests.gpu_util import slice_rel_max, tube_rel_max

    cmp = {}
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    m_obs = np.asarray(w["M_obs"], dtype=np.float64)
    c = cases["video"]
    t0 = time.perf_counter()
    ref = admm.complete(m_obs, w["mask"], w["rho"], w["growth"], w["rho_max"], max_iter=c["iters"], tol=0.0)["X"]
    dt = time.perf_counter() - t0
    den = np.linalg.norm(ref)
    cmp["parity"] = {"iters": c["iters"], "what": "the timed GPU runs' outputs against the oracle, same iterations",
                     "fp64_rel_err_vs_oracle": float(np.linalg.norm(c["got64"] - ref) / den),
                     "fp32_rel_err_vs_oracle": float(np.linalg.norm(c["got32"] - ref) / den),
                     "fp32_slice_max_rel_err": slice_rel_max(c["got32"], ref),
                     "fp32_tube_max_rel_err": tube_rel_max(c["got32"], ref),
                     "fp64_bar": 1e-10, "fp32_bar": 1e-4}
    with threadpool_limits(limits=1):
        t1 = time.perf_counter()
        admm.complete(m_obs, w["mask"], w["rho"], w["growth"], w["rho_max"], max_iter=single_iters, tol=0.0)
        dt1 = time.perf_counter() - t1
    cpu_model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), cpu_model)
    except OSError:
        pass
    base = dict(value=c["iters"] / dt, unit="iters/s", cores=threads, kind="oracle",
                cpu_model=cpu_model, nproc=os.cpu_count(),
                sample=f"the same {c['iters']} ADMM iterations of the 128x160x64 completion as the timed GPU steps "
                       f"({dt:.1f} s, NumPy FP64, BLAS threads={threads})",
                single_core={"value": single_iters / dt1, "unit": "iters/s", "cores": 1,
                             "sample": f"first {single_iters} iterations, BLAS threads=1 ({dt1:.1f} s)"})
    if "serving" in cases:
        # the serving mix is not served on the host: the oracle's solve time
        # per request instead, from two timed iterations of each of the first
        # requests, scaled to the iterations the GPU leg ran on average
        c = cases["serving"]
        per_iter, solve = [], []
        for d in c["requests"]:
            t2 = time.perf_counter()
            if d["kind"] == "complete":
                admm.complete(d["M_obs"], d["mask"], d["rho"], d["growth"], d["rho_max"], max_iter=2, tol=0.0)
            else:
                admm.trpca(d["M"], d["lam"], d["mu"], d["growth"], d["mu_max"], max_iter=2, tol=0.0)
            pi = (time.perf_counter() - t2) / 2
            per_iter.append(pi)
            solve.append(pi * c["iters"])
        solve = np.asarray(solve)
        base["serving_oracle"] = {
            "requests": len(solve), "iters_per_request": c["iters"],
            "solve_s_p50": float(np.percentile(solve, 50)), "solve_s_max": float(solve.max()),
            "per_iter_s": [round(x, 4) for x in per_iter],
            "sample": "the first requests of the 50 req/s trace, 2 oracle iterations each, scaled"}
    if "batched" in cases:
        c = cases["batched"]
        d = c["data"]
        ref = admm.complete(d["M_obs"], d["mask"], d["rho"], d["growth"], d["rho_max"], max_iter=c["iters"],
                            tol=0.0)["X"]
        cmp["batched_sampled_rse_vs_oracle"] = float(np.linalg.norm(c["got"] - ref) / np.linalg.norm(ref))
    if "sweep" in cases:
        c = cases["sweep"]
        ref = admm.complete(c["y"], c["mask"], c["rho"], c["growth"], c["rho_max"], max_iter=c["iters"],
                            tol=0.0)["X"]
        cmp["sweep_matrix_baseline_rel_err_vs_oracle"] = float(np.linalg.norm(c["got"] - ref) / np.linalg.norm(ref))
    if "tube_rpca" in cases:
        c = cases["tube_rpca"]
        n1, n2, n3 = c["m"].shape
        errs = {}
        for name, x, lam, shrink in (("tensor", c["m"], c["lam_tensor"], "l112"),
                                     ("matrix", c["m"].reshape(n1 * n2, n3, 1), c["lam_matrix"], "l1")):
            ref = admm.trpca(x, lam, c["mu"], c["growth"], c["mu_max"], max_iter=c["iters"], tol=0.0, shrink=shrink)
            got_l, got_s = c["got_" + name]
            errs[name + "_l_rel_err_vs_oracle"] = float(
                np.linalg.norm(got_l.reshape(x.shape) - ref["L"]) / np.linalg.norm(ref["L"]))
            errs[name + "_s_rel_err_vs_oracle"] = float(
                np.linalg.norm(got_s.reshape(x.shape) - ref["S"]) / max(np.linalg.norm(ref["S"]), 1e-300))
        cmp["tube_rpca"] = errs
    if "compression" in cases:
        c = cases["compression"]
        t0 = time.perf_counter()
        otensor.tsvd(c["x"])
        t_tsvd = time.perf_counter() - t0
        ref = ocompress.method1(c["x"], c["k2"])
        cmp["compression"] = {"method1_k2": c["k2"],
                              "method1_rel_err_vs_oracle": float(np.linalg.norm(c["got"] - ref) / np.linalg.norm(ref)),
                              "oracle_tsvd_ms": t_tsvd * 1e3}
    return base, cmp


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-single-iters", type=int, default=10,
                    help="oracle iterations timed with one BLAS thread")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--only", choices=["fp32", "fp64"], default=None,
                    help="run one form only (for profiler runs); prints its timing line")
    ap.add_argument("--batch-iters", type=int, default=150, help="iterations per batched problem")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-compress", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-tube-rpca", action="store_true")
    ap.add_argument("--no-trpca256", action="store_true")
    ap.add_argument("--sweep-iters", type=int, default=150)
    ap.add_argument("--serve-rate", type=float, default=50.0)
    ap.add_argument("--serve-window", type=float, default=4.0,
                    help="seconds of arrivals replayed: the first 4 s of the 60-s trace by default, since "
                         "the trace's 3000 requests at ~12 solves/s would take about four minutes to drain")
    ap.add_argument("--serve-limit", type=float, default=240.0,
                    help="wall-clock limit of a serving window; open requests are then cancelled")
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--serve-sustained-rate", type=float, default=2.0,
                    help="second serving window at a rate below capacity (0: skip)")
    ap.add_argument("--serve-sustained-window", type=float, default=10.0)
    ap.add_argument("--only-legs", action="store_true", help="run the batched and serving legs only")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain device copy of 1 GiB (reference for HBM byte counters) and exit")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
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
    if args.only_legs:
        res = {}
        if not args.no_batch:
            res["batched"], _ = batched_leg(lib, torch, np, workloads, args.batch_iters)
            print(json.dumps({"batched": res["batched"]}), flush=True)
        if not args.no_serve:
            res["serving"] = serving_leg(lib, torch, np, workloads, args.serve_rate, args.serve_window,
                                         args.serve_budget_gb, args.serve_limit)
            print(json.dumps({"serving": res["serving"]}), flush=True)
            if args.serve_sustained_rate > 0:
                res["serving_sustained"] = serving_leg(lib, torch, np, workloads, args.serve_sustained_rate,
                                                       args.serve_sustained_window, args.serve_budget_gb,
                                                       args.serve_limit)
                print(json.dumps({"serving_sustained": res["serving_sustained"]}), flush=True)
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

    m_dim, n_dim = max(SHAPE[0], SHAPE[1]), min(SHAPE[0], SHAPE[1])
    h_dim = SHAPE[2] // 2 + 1
    if not args.no_profile:
        copy_gbs = device_copy_gbs(torch)
        handle.profile(True)
        lib.tsvd_complete(obs32, mask, max_iter=args.steps, **kw, **fp32)
        handle.profile(False)
        stats = handle.profile_read()
        result["roofline"] = roofline(stats, True, m_dim, n_dim)
        result["side_rooflines"] = side_rooflines(stats, True, m_dim, n_dim, h_dim, copy_gbs)
        result["kernels_ms_per_step"] = {k: v["total_ms"] / args.steps for k, v in stats.items()}
        handle.profile(True)
        lib.tsvd_complete(obs64, mask, max_iter=args.steps, **kw)
        handle.profile(False)
        stats64 = handle.profile_read()
        result["fp64_plain"]["roofline"] = roofline(stats64, False, m_dim, n_dim)
        result["fp64_plain"]["side_rooflines"] = side_rooflines(stats64, False, m_dim, n_dim, h_dim, copy_gbs)

    # the timed runs' outputs, compared with the oracle at the same iteration count by the CPU leg
    cases = {"video": {"iters": args.steps, "got64": x64n, "got32": x32.cpu().numpy().astype(np.float64)}}

    if not args.no_batch:
        result["batched"], cases["batched"] = batched_leg(lib, torch, np, workloads, args.batch_iters)
    if not args.no_compress:
        result["compression"], cases["compression"] = compression_leg(lib, torch, np, workloads)
    if not args.no_sweep:
        result["sampling_sweep"], cases["sweep"] = sweep_leg(lib, torch, np, workloads, args.sweep_iters)
    if not args.no_tube_rpca:
        result["tube_rpca"], cases["tube_rpca"] = tube_rpca_leg(lib, torch, np, workloads)
    if not args.no_trpca256:
        result["trpca_256"] = trpca_256_leg(lib, torch, np, workloads)
        print("[bench] trpca 256 leg done", file=sys.stderr, flush=True)
    if not args.no_serve:
        result["serving"] = serving_leg(lib, torch, np, workloads, args.serve_rate, args.serve_window,
                                        args.serve_budget_gb, args.serve_limit)
        result["serving"]["trace_cap"] = (f"first {args.serve_window:g} s of the 60-s trace: at the engine's "
                                          "capacity the full trace would take about four minutes to drain")
        cases["serving"] = {"requests": [workloads.serve_request(r)
                                         for r in workloads.arrivals(0, args.serve_rate, args.serve_window)[:6]],
                            "iters": max(1, int(round(result["serving"]["mean_iters"])))}
        if args.serve_sustained_rate > 0:
            # below capacity: latency is the service time in the mix, not queueing
            result["serving_sustained"] = serving_leg(lib, torch, np, workloads, args.serve_sustained_rate,
                                                      args.serve_sustained_window, args.serve_budget_gb,
                                                      args.serve_limit)
    if not args.no_cpu_baseline:
        print("[bench] cpu leg", file=sys.stderr, flush=True)
        result["cpu_baseline"], cmp = cpu_baseline(w, cases, args.cpu_single_iters)
        result["parity"] = cmp.get("parity")
        if "batched" in result:
            result["batched"]["sampled_rse_vs_oracle"] = cmp.get("batched_sampled_rse_vs_oracle")
        if "compression" in result:
            result["compression"].update(cmp.get("compression", {}))
        if "tube_rpca" in result:
            result["tube_rpca"]["prefix_vs_oracle"] = cmp.get("tube_rpca")
        if "sampling_sweep" in result:
            result["sampling_sweep"]["matrix_baseline_prefix_rel_err_vs_oracle"] = cmp.get(
                "sweep_matrix_baseline_rel_err_vs_oracle")
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
