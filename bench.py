"""Benchmark of the Galerkin-FFT Newton--CG hot path on one MI355X.

One step = one full solve of the workload's mean-strain path (every
increment of Algorithm 1: return map, residual G:sigma, CG with the
matrix-free G:(C:p) product, Newton updates, history commit) from a fresh
history, inputs already resident in HBM.  The metric is
voxel-CG-iterations per second: voxels x CG iterations of the timed steps
divided by their wall time.

Default workload: the 31^3 Bernoulli(0.3) two-phase RVE in FP64, pure shear
E_eq = 0.02 in 10 increments.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

HBM_PEAK_GBS = 8000.0


WORKLOADS = {
    "random_31": "31^3 Bernoulli(0.3) two-phase J2 RVE, FP64, pure shear 0.02 in 10 increments",
    "voronoi_127_mixed": "127^3 periodic Voronoi (200 grains, 20% hard), FP32 product / FP64 rest, 20 increments",
    "voronoi_127_fp64": "127^3 periodic Voronoi (200 grains, 20% hard), FP64, 20 increments",
    "batch64_fp64": "64 RVEs, N in {15,31,63}, hard fraction U[0.1,0.5], yield contrast U[1.5,4], FP64, 10 increments, one batched launch per pass",
    "batch64_mixed": "64 RVEs as batch64_fp64 with the FP32 product",
}


def workload(name: str):
    """List of synth.Workload for the named benchmark configuration."""
    if name == "random_31":
        return [synth.random_31()]
    if name == "voronoi_127_mixed":
        return [synth.voronoi_127(precision="mixed")]
    if name == "voronoi_127_fp64":
        return [synth.voronoi_127(precision="fp64")]
    if name == "batch64_fp64":
        return synth.batch_64(precision="fp64")
    if name == "batch64_mixed":
        return synth.batch_64(precision="mixed")
    raise SystemExit(f"unknown workload {name}")


def tensor6(E):
    return [E[0, 0], E[1, 1], E[2, 2], E[1, 2], E[0, 2], E[0, 1]]


def x_pass_bytes_per_voxel(shape, real_bytes):
    """Algorithmic HBM bytes of one x-pass launch per voxel: it reads and
    writes the six complex half-spectrum planes once (n0*n1*H complex each)."""
    n0, n1, n2 = shape
    H = (n2 + 1) // 2
    return 2 * 6 * 2 * real_bytes * (n0 * n1 * H) / float(n0 * n1 * n2)


def forward_pass_bytes_per_voxel(shape, real_bytes):
    """Algorithmic HBM bytes per voxel of one forward product pass inside CG
    (k_zfwd or k_slab_fwd): read r and p (6 FP64 each), the compact tangent
    (7 reals of the apply precision) and the phase byte; write the new p (6
    FP64) and the six complex half-spectrum planes.  The y transform of the
    slab form stays in LDS and adds no HBM bytes."""
    n0, n1, n2 = shape
    H = (n2 + 1) // 2
    return 6 * 8 * 3 + 7 * real_bytes + 1 + 6 * 2 * real_bytes * H / float(n2)


ROOFLINE_KERNELS = {
    0: ("forward product pass k_zfwd (k_slab_fwd with the fused slab passes): p <- r + beta p, C:p, "
        "DFT along z (and y)", forward_pass_bytes_per_voxel),
    2: ("k_xpass (DFT x, G^(k) projection, inverse DFT x)", x_pass_bytes_per_voxel),
}


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "fft_lds.h", "fftg_internal.h", "radix_consts.h"):
        with open(os.path.join(ROOT, "paper_1601_05970_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload_name, kernel_id):
    """HBM bytes per launch of the roofline kernel from the committed
    FETCH_SIZE/WRITE_SIZE summary, or None when it covers another workload,
    another kernel or older kernel sources."""
    path = os.path.join(ROOT, "profiles", "random31_fp64_hbm_traffic.md")
    if workload_name != "random_31" or not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith(("#", "|", "`")):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_source_hash() or kv.get("kernel_id") != str(kernel_id):
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(w, budget_s=15.0):
    """The FP64 oracle on the host cores, increments 1.. until ~budget_s."""
    from oracle import solver as S
    s = S.Solver(w.phase, w.materials, w.tol_newton, w.tol_cg)
    t0 = time.perf_counter()
    cg = 0
    n = 0
    while n < w.n_inc and time.perf_counter() - t0 < budget_s:
        n += 1
        cg += sum(s.solve_increment(w.E_at(n)).cg_iters)
    dt = time.perf_counter() - t0
    return {"value": w.nvox * cg / dt, "unit": "voxel-CG-iters/s", "cores": os.cpu_count(), "kind": "oracle",
            "sample": f"{w.name}: increments 1-{n} of {w.n_inc} ({cg} CG iterations, {dt:.1f} s), numpy/scipy "
                      f"FP64, scipy.fft workers=all cores"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="random_31")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-kernel", type=int, default=0, choices=sorted(ROOFLINE_KERNELS),
                    help="fftg_kernel_id timed for the roofline (0: forward product pass, 2: x pass)")
    ap.add_argument("--profile-every", type=int, default=16,
                    help="bracket one launch in this many of the roofline kernel with timing events")
    ap.add_argument("--also", default="batch64_fp64,batch64_mixed",
                    help="extra workloads timed after the main one (1 warmup + 1 step each); '' for none")
    ap.add_argument("--max-increments", type=int, default=0,
                    help="profiling runs only: stop each solve after this many increments")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a device copy of MIB MiB 10 times (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the solve of one RVE is not sharded "
              "across GPUs by this library", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1601_05970_amd import fftg

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch_read": n * 8, "copy_bytes_per_launch_write": n * 8, "launches": 10}))
        return

    result = measure(fftg, torch, args.workload, args.steps, args.warmup, args.profile_kernel, args.max_increments,
                     args.profile_every)
    out = result
    out["n_gpus"] = 1
    if not args.no_cpu_baseline:
        ws = workload(args.workload)
        out["cpu_baseline"] = cpu_baseline(ws[0] if len(ws) == 1 else max(ws, key=lambda x: x.nvox))
    also = [a for a in args.also.split(",") if a and a != args.workload]
    if also:
        out["also"] = []
        for name in also:
            r = measure(fftg, torch, name, 1, 1, args.profile_kernel, 0, args.profile_every)
            out["also"].append({"workload": r["config"]["workload"], "value": r["value"], "unit": r["unit"],
                                "dtype": r["dtype"], "ms_per_step": r["ms_per_step"],
                                "rves": r["config"]["rves"], "voxels": r["config"]["voxels"],
                                "roofline_frac": r["roofline"]["frac"],
                                "roofline_kernel_GBs": r["roofline"]["achieved"]})
    print(json.dumps(out))


def measure(fftg, torch, name, steps, warmup, profile_kernel, max_inc=0, profile_every=16):
    """Times `steps` full solves of workload `name`; returns the bench dict."""
    ws = workload(name)
    if max_inc:
        for x in ws:
            x.E_final = x.E_final * (min(max_inc, x.n_inc) / x.n_inc)
            x.n_inc = min(max_inc, x.n_inc)
    desc = WORKLOADS[name]
    w = ws[0]
    opts = fftg.fftg_options_default()
    opts.tol_newton, opts.tol_cg = w.tol_newton, w.tol_cg
    opts.precision = fftg.FFTG_MIXED if w.precision == "mixed" else fftg.FFTG_FP64
    plans = [fftg.Plan(x.phase, x.materials, opts) for x in ws]
    nvox = np.array([x.nvox for x in ws], dtype=np.float64)

    def step():
        """One full solve of every RVE's load path from a fresh history;
        returns the CG iterations of each RVE."""
        hs = [fftg.History(p) for p in plans]
        cg = np.zeros(len(ws))
        if len(ws) == 1:
            for n in range(1, w.n_inc + 1):
                cg[0] += hs[0].solve_increment(tensor6(w.dE(n)))["total_cg"]
        else:
            batch = fftg.Batch(plans, hs)
            for n in range(1, w.n_inc + 1):
                dE = np.array([tensor6(x.dE(n)) for x in ws])
                st = batch.solve_increment(dE)
                cg += np.array([s["total_cg"] for s in st], dtype=np.float64)
            batch.close()
        for h in hs:
            h.close()
        return cg

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # one launch in profile_every is bracketed by timing events: each pair adds
    # a few microseconds of queue processing between kernels, which at 31^3 is
    # a fifth of a CG iteration when every launch is bracketed
    fftg.fftg_profiler_start_every(profile_kernel, profile_every)
    t0 = time.perf_counter()
    cg_iters = np.zeros(len(ws))
    for _ in range(steps):
        cg_iters += step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kms, klaunch, kvox = fftg.fftg_profiler_stop()
    kseen = fftg.fftg_profiler_seen()

    total_work = float(np.dot(nvox, cg_iters))
    value = total_work / dt
    real_bytes = 4 if opts.precision == fftg.FFTG_MIXED else 8
    kname, kbytes = ROOFLINE_KERNELS[profile_kernel]
    # Algorithmic bytes of the timed launches, counted from the work done: each
    # CG iteration of an RVE moves its per-voxel bytes once through the kernel
    # (in a batch, RVEs whose CG has stopped exit their tiles at once, so the
    # launch count alone would overstate the bytes).  The kernel's few launches
    # outside CG (residual, predictor) add time but are not counted: the
    # achieved rate is a lower bound.
    # The kernel time of all launches is the sampled average times their count.
    total_bytes = float(np.dot(nvox * cg_iters, [kbytes(x.shape, real_bytes) for x in ws]))
    avg_ms = kms / max(klaunch, 1)
    bytes_per_launch = total_bytes / max(kseen, 1)
    achieved = total_bytes / (avg_ms * kseen * 1e-3) / 1e9 if kms > 0 else 0.0
    for p in plans:
        p.close()
    return {
        "metric": "voxel-CG-iters/s", "value": value, "unit": "voxel-CG-iters/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": 1e3 * dt / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if opts.precision == fftg.FFTG_MIXED else "f64", "data": "synthetic",
        "config": {"workload": desc, "rves": len(ws), "voxels": int(nvox.sum()),
                   "grid": list(w.shape) if len(ws) == 1 else "mixed", "increments": w.n_inc,
                   "tol_newton": w.tol_newton, "tol_cg": w.tol_cg,
                   "voxel_cg_iters_per_step": total_work / steps},
        "roofline": {"kernel": kname, "bound": "hbm",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(name, profile_kernel),
                     "avg_launch_us": 1e3 * avg_ms, "launches": kseen, "timed_launches": klaunch,
                     "bytes_per_launch": bytes_per_launch},
    }


if __name__ == "__main__":
    main()
