"""Benchmark of the Galerkin-FFT Newton--CG hot path on one MI355X.

Headline workload: the 64-RVE batch (N drawn from {15, 31, 63}, random
two-phase J2 microstructures, pure shear E_eq = 0.02 in 10 increments), FP64,
every launch covering all members.  One step is one increment of the batch's
load path for every member -- all rows of the hot path: return map and
consistent tangent, residual G:sigma, CG with the matrix-free G:(C:p) product,
Newton updates, history commit -- with inputs resident in HBM.  The load path
restarts from fresh histories after its last increment (histories and the
batch are created before the timed region), so 20 timed steps after 5 warm-up
steps cover every increment of the path exactly twice.  The metric is
voxel-CG-iterations per second: voxels x CG iterations of the timed steps
divided by their wall time.

The JSON line also carries (`also`) the batch with the FP32 product, the
127^3 Voronoi RVE in FP64 and in mixed precision (one full 20-increment solve
each, with the mixed solve's relative error against the FP64 one) and the
31^3 RVE in FP64; the roofline of the dominant product pass and of the whole
CG iteration, timed live with HIP events; a measured device copy as the
attainable-bandwidth line; and the FP64 oracle on the host cores.
"""
from __future__ import annotations

import argparse
import json
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
    "batch64_fp64": "64 RVEs, N in {15,31,63}, hard fraction U[0.1,0.5], yield contrast U[1.5,4], FP64, "
                    "10 increments, every launch covering all members",
    "batch64_mixed": "64 RVEs as batch64_fp64 with the FP32 product",
}

# kernel kinds of the product passes (fftg_kernel_id) and their names
PASSES = {0: "k_zfwd", 1: "k_ypass fwd", 2: "k_xpass", 3: "k_ypass inv", 4: "k_zinv"}
SLAB_NAMES = {0: "k_slab_fwd", 2: "k_xpass", 4: "k_slab_inv"}


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


def pass_bytes_per_voxel(kid, shape, real_bytes, slab):
    """Algorithmic HBM bytes per voxel of one launch of a product pass inside
    CG (s = real_bytes of the apply precision; CG vectors are FP64; H/n2 of
    the half spectrum):
      forward  (k_zfwd / k_slab_fwd): read r, p (6 FP64 each), the compact
               tangent (7 s) and the phase byte; write p and the half
               spectrum (6 complex s x H/n2);
      y pass   (five passes only): read and write the half spectrum;
      x pass:  read and write the half spectrum (G^ applied between the
               transforms, in LDS);
      inverse  (k_zinv / k_slab_inv): read the half spectrum, x, r and p;
               write x and r.
    The slab passes keep the y transforms in LDS, so they move no more than
    the z passes."""
    n0, n1, n2 = shape
    h = ((n2 + 1) // 2) / float(n2)
    spec = 6 * 2 * real_bytes * h
    if kid == 0:
        return 6 * 8 * 3 + 7 * real_bytes + 1 + spec
    if kid in (1, 3):
        return 0.0 if slab else 2 * spec
    if kid == 2:
        return 2 * spec
    if kid == 4:
        return spec + 6 * 8 * 5
    raise ValueError(kid)


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "fft_lds.h", "fftg_internal.h", "radix_consts.h"):
        with open(os.path.join(ROOT, "paper_1601_05970_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload_name):
    """Per-kind HBM bytes per launch from the committed FETCH_SIZE/WRITE_SIZE
    summary of this workload, or {} when there is none or it was taken on
    other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{workload_name}_hbm_traffic.md")
    if not os.path.exists(path):
        return {}
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith(("#", "|", "`", " ", "-")):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_source_hash():
        return {}
    out = {}
    for kid in PASSES:
        v = kv.get(f"traffic_bytes_per_launch_kind{kid}")
        if v is not None:
            try:
                out[kid] = float(v)
            except ValueError:
                pass
    return out


def cpu_baseline(w, budget_s=15.0):
    """The FP64 oracle on the host cores, increments 1.. of w until ~budget_s."""
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
            "sample": f"{w.name} ({'x'.join(map(str, w.shape))}): increments 1-{n} of {w.n_inc} ({cg} CG "
                      f"iterations, {dt:.1f} s), numpy/scipy FP64, scipy.fft workers=all cores"}


def device_copy_gbs(torch, mib=1024, reps=10):
    """Attainable-bandwidth line: a device-to-device copy of mib MiB, read +
    write bytes over the event-timed duration."""
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    b.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * n * 8 / (ms * 1e-3) / 1e9


class Runner:
    """Plans of a workload and the load path split into steps of one
    increment; histories (and the batch over them) for every load path the
    run needs are created up front."""

    def __init__(self, fftg, name, n_paths, max_inc=0):
        self.fftg = fftg
        self.ws = workload(name)
        if max_inc:
            for x in self.ws:
                x.E_final = x.E_final * (min(max_inc, x.n_inc) / x.n_inc)
                x.n_inc = min(max_inc, x.n_inc)
        w = self.ws[0]
        self.w = w
        opts = fftg.fftg_options_default()
        opts.tol_newton, opts.tol_cg = w.tol_newton, w.tol_cg
        opts.precision = fftg.FFTG_MIXED if w.precision == "mixed" else fftg.FFTG_FP64
        self.opts = opts
        self.plans = [fftg.Plan(x.phase, x.materials, opts) for x in self.ws]
        self.nvox = np.array([x.nvox for x in self.ws], dtype=np.float64)
        self.paths = []
        for _ in range(n_paths):
            hs = [fftg.History(p) for p in self.plans]
            b = fftg.Batch(self.plans, hs) if len(self.ws) > 1 else None
            self.paths.append((hs, b))
        self.k = 0   # steps taken
        self.sigma = []  # Sigma of every member after each increment of the current path

    @property
    def n_inc(self):
        return self.w.n_inc

    def step(self):
        """One increment for every member; returns the CG iterations of each."""
        path, n = divmod(self.k, self.n_inc)
        n += 1
        hs, b = self.paths[path]
        self.k += 1
        if n == 1:
            self.sigma = []
        if b is None:
            st = [hs[0].solve_increment(tensor6(self.w.dE(n)))]
        else:
            st = b.solve_increment(np.array([tensor6(x.dE(n)) for x in self.ws]))
        self.sigma.append([s["Sigma"] for s in st])
        self.last = st
        return np.array([s["total_cg"] for s in st], dtype=np.float64)

    def strain(self, path):
        """Strain fields of every member at the end of a load path (host)."""
        hs, _ = self.paths[path]
        return [h.get_field(self.fftg.FFTG_FIELD_STRAIN).cpu().numpy() for h in hs]

    def close(self):
        for hs, b in self.paths:
            if b is not None:
                b.close()
            for h in hs:
                h.close()
        for p in self.plans:
            p.close()


def measure(fftg, torch, name, steps, warmup, max_inc=0, profile_every=16, keep=False):
    """Times `steps` increments of workload `name` after `warmup` (steps of
    None: one full load path after one warm-up path).  Returns the bench
    dict, and the runner when keep is set."""
    probe = workload(name)
    n_inc = min(max_inc, probe[0].n_inc) if max_inc else probe[0].n_inc
    if steps is None:
        steps, warmup = n_inc, n_inc
    n_paths = (warmup + steps + n_inc - 1) // n_inc
    r = Runner(fftg, name, n_paths, max_inc)
    for _ in range(warmup):
        r.step()
    torch.cuda.synchronize()
    # one launch in profile_every of every product pass is bracketed by timing
    # events on the stream it runs on
    fftg.fftg_profiler_start_set(list(PASSES), profile_every)
    t0 = time.perf_counter()
    cg = np.zeros(len(r.ws))
    for _ in range(steps):
        cg += r.step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    fftg.fftg_profiler_stop()
    kinds = {k: fftg.fftg_profiler_kind(k) for k in PASSES}
    mixed = r.opts.precision == fftg.FFTG_MIXED
    real_bytes = 4 if mixed else 8
    slab = kinds[1][3] == 0   # the slab schedule runs no y passes
    work = float(np.dot(r.nvox, cg))
    # per pass: algorithmic bytes of the CG iterations done (each iteration of
    # an RVE moves its per-voxel bytes once through the pass; members whose CG
    # has stopped exit their tiles at once), and the pass's time over all its
    # launches = sampled average x launch count.  Launches outside CG
    # (residual, predictor, equilibrium) add time but no counted bytes, so the
    # rates are lower bounds.
    passes = {}
    tot_bytes = tot_ms = 0.0
    for kid in PASSES:
        ms, nb, _, seen = kinds[kid]
        if seen == 0:
            continue
        bpv = np.array([pass_bytes_per_voxel(kid, x.shape, real_bytes, slab) for x in r.ws])
        byt = float(np.dot(r.nvox * cg, bpv))
        t_ms = ms / max(nb, 1) * seen
        passes[kid] = {"kernel": (SLAB_NAMES if slab else PASSES)[kid], "avg_launch_us": 1e3 * ms / max(nb, 1),
                       "launches": seen, "timed_launches": nb, "bytes_per_launch": byt / seen,
                       "achieved_GBs": byt / (t_ms * 1e-3) / 1e9 if t_ms > 0 else 0.0, "ms_total": t_ms}
        tot_bytes += byt
        tot_ms += t_ms
    dom = max(passes, key=lambda k: passes[k]["ms_total"])
    res = {
        "metric": "voxel-CG-iters/s", "value": work / dt, "unit": "voxel-CG-iters/s", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": 1e3 * dt / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64", "data": "synthetic",
        "config": {"workload": WORKLOADS[name], "rves": len(r.ws), "voxels": int(r.nvox.sum()),
                   "grid": list(r.w.shape) if len(r.ws) == 1 else "mixed", "increments": n_inc,
                   "step": "one increment of the load path for every RVE",
                   "tol_newton": r.w.tol_newton, "tol_cg": r.w.tol_cg, "schedule": "slab" if slab else "five-pass",
                   "voxel_cg_iters_per_step": work / steps},
        "passes": passes, "dominant": dom, "product_bytes": tot_bytes, "product_ms": tot_ms,
    }
    if keep:
        return res, r
    r.close()
    return res


def product_bytes_per_voxel(shape, real_bytes):
    """Algorithmic HBM bytes per voxel of one fftg_apply_GK in the five-pass
    schedule: read the FP64 input and the phase byte, write the output (apply
    precision), and move the half spectrum (6 complex values of s bytes x
    H/n2 per voxel) eight times: written by the z pass, read and written by
    the y, x and inverse y passes, read by the inverse z pass."""
    n0, n1, n2 = shape
    spec = 6 * 2 * real_bytes * ((n2 + 1) // 2) / float(n2)
    return 6 * 8 + 1 + 6 * real_bytes + 8 * spec


def time_products(fftg, torch, sizes, reps=20):
    """Event-timed back-to-back products on N^3 two-phase grids."""
    out = {"products": []}
    for n in sizes:
        shape = (n, n, n)
        ph = synth.bernoulli(shape, 0.3, 1)
        p = torch.randn((6,) + shape, dtype=torch.float64, device="cuda")
        for prec, name, dt in ((fftg.FFTG_FP64, "fp64", torch.float64), (fftg.FFTG_MIXED, "fp32", torch.float32)):
            opt = fftg.fftg_options_default()
            opt.precision = prec
            pl = fftg.Plan(ph, [synth.SOFT, synth.HARD], opt)
            o = torch.empty((6,) + shape, dtype=dt, device="cuda")
            pl.apply_GK(p, o, fftg.FFTG_TANGENT_ELASTIC)   # autotunes
            torch.cuda.synchronize()
            fftg.fftg_profiler_start_set(list(PASSES), 1)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                pl.apply_GK(p, o, fftg.FFTG_TANGENT_ELASTIC)
            b.record()
            b.synchronize()
            fftg.fftg_profiler_stop()
            us = 1e3 * a.elapsed_time(b) / reps
            byt = product_bytes_per_voxel(shape, 4 if prec else 8) * n ** 3
            item = {"N": n, "precision": name, "us_per_product": us, "GBs": byt / (us * 1e-6) / 1e9,
                    "frac": byt / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, "bytes_per_voxel": byt / n ** 3, "passes_us": {}}
            for kid in PASSES:
                ms, nb, _, seen = fftg.fftg_profiler_kind(kid)
                if nb:
                    item["passes_us"][PASSES[kid]] = 1e3 * ms / nb
            out["products"].append(item)
            del o, pl
            torch.cuda.empty_cache()
        del p
    return out


def rel_err(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(float(np.max(np.abs(b))), 1e-300))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed increments of the load path")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="batch64_fp64", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-every", type=int, default=16,
                    help="bracket one launch in this many of each product pass with timing events")
    ap.add_argument("--also", default="batch64_mixed,voronoi_127_fp64,voronoi_127_mixed,random_31",
                    help="extra workloads, one full load path each after a warm-up; '' for none")
    ap.add_argument("--max-increments", type=int, default=0,
                    help="profiling runs only: cut each load path to this many increments")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a device copy of MIB MiB 10 times (HBM counter calibration) and exit")
    ap.add_argument("--serve", type=int, default=24, metavar="REQUESTS",
                    help="served stream after the solves: this many requests of the serving recipe (sizes "
                         "--serve-sizes), saturated and then Poisson at 0.8x the saturated rate; 0 for none")
    ap.add_argument("--serve-sizes", default="31,63,127")
    ap.add_argument("--products", default="", metavar="N,N,...",
                    help="only time the product G:(Ce:p) (fftg_apply_GK, ELASTIC) on N^3 grids in FP64 and FP32 "
                         "and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): RVEs are not sharded across GPUs by "
              "this library", file=sys.stderr)
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

    if args.products:
        print(json.dumps(time_products(fftg, torch, [int(n) for n in args.products.split(",")])))
        return

    copy_gbs = device_copy_gbs(torch)
    out, runner = measure(fftg, torch, args.workload, args.steps, args.warmup, args.max_increments,
                          args.profile_every, keep=True)
    traffic = measured_traffic(args.workload)
    dom = out.pop("dominant")
    passes = out.pop("passes")
    pb, pms = out.pop("product_bytes"), out.pop("product_ms")
    d = passes[dom]
    out["roofline"] = {
        "kernel": d["kernel"], "bound": "hbm", "achieved": d["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": d["achieved_GBs"] / HBM_PEAK_GBS, "traffic": traffic.get(dom),
        "avg_launch_us": d["avg_launch_us"], "launches": d["launches"], "timed_launches": d["timed_launches"],
        "bytes_per_launch": d["bytes_per_launch"],
        "attainable_copy_GBs": copy_gbs,
        "product": {"kernels": [passes[k]["kernel"] for k in passes], "achieved": pb / (pms * 1e-3) / 1e9,
                    "frac": pb / (pms * 1e-3) / 1e9 / HBM_PEAK_GBS, "bytes": pb, "ms": pms},
        "passes": {passes[k]["kernel"]: {"achieved": passes[k]["achieved_GBs"], "avg_launch_us": passes[k]["avg_launch_us"],
                                         "bytes_per_launch": passes[k]["bytes_per_launch"],
                                         "traffic": traffic.get(k)} for k in passes},
    }
    # FP64 reference of the mixed batch: Sigma after each increment of the
    # last complete load path and the final strain fields
    ref = None
    if runner.k >= runner.n_inc:
        last = runner.k // runner.n_inc - 1
        ref = {"strain": runner.strain(last)}
    runner.close()
    if not args.no_cpu_baseline:
        ws = workload(args.workload)
        out["cpu_baseline"] = cpu_baseline(ws[0] if len(ws) == 1 else max(ws, key=lambda x: x.nvox))
    also = [a for a in args.also.split(",") if a and a != args.workload]
    if also:
        out["also"] = []
        fp64_127 = None
        for name in also:
            r, run = measure(fftg, torch, name, None, None, args.max_increments, args.profile_every, keep=True)
            item = {"workload": r["config"]["workload"], "value": r["value"], "unit": r["unit"], "dtype": r["dtype"],
                    "ms_per_path": r["ms_per_step"] * r["steps"],
                    "timed": "one full load path (all increments) after a warm-up path", "rves": r["config"]["rves"],
                    "voxels": r["config"]["voxels"], "schedule": r["config"]["schedule"],
                    "product_GBs": r["product_bytes"] / (r["product_ms"] * 1e-3) / 1e9,
                    "dominant_pass": r["passes"][r["dominant"]]["kernel"],
                    "dominant_GBs": r["passes"][r["dominant"]]["achieved_GBs"]}
            item["product_frac"] = item["product_GBs"] / HBM_PEAK_GBS
            # relative error of the mixed solves against FP64 solves of the same
            # RVEs at the same (configured) tolerances: Sigma over the load path
            # and the final local strain field
            if name == "voronoi_127_fp64":
                fp64_127 = {"sigma": np.array(run.sigma), "strain": run.strain(1)}
            if name == "voronoi_127_mixed" and fp64_127 is not None:
                item["vs_fp64"] = {"Sigma_rel_err": rel_err(run.sigma, fp64_127["sigma"]),
                                   "strain_rel_err": rel_err(run.strain(1)[0], fp64_127["strain"][0])}
            if name == "batch64_mixed" and ref is not None and args.workload == "batch64_fp64":
                st = run.strain(1)
                item["vs_fp64"] = {"strain_rel_err_max_over_rves": max(rel_err(a, b) for a, b in zip(st, ref["strain"]))}
            run.close()
            out["also"].append(item)
    if args.serve:
        out["serving"] = serve_stream(torch, args.serve, [int(n) for n in args.serve_sizes.split(",")])
    print(json.dumps(out))


def serve_stream(torch, n_requests, sizes, rate_factor=0.8):
    """The continuous-batching server on a stream of the serving recipe
    (Voronoi RVEs of the listed sizes with the recipe's weights renormalised,
    50-400 grains, 5-20 increments, FP64 or mixed at 50/50): first with every
    request present at t = 0 (saturated throughput), then with Poisson
    arrivals at rate_factor x that throughput; latency = completion - arrival."""
    from paper_1601_05970_amd.serve import FftgExecutor, Server, summarize
    allw = {31: 0.4, 63: 0.3, 127: 0.2, 255: 0.1}
    wts = np.array([allw[n] for n in sizes])
    wts = tuple(float(x) for x in wts / wts.sum())
    free, _ = torch.cuda.mem_get_info()
    ex = FftgExecutor()
    base = synth.serving_stream(n_requests, rate=1e9, sizes=tuple(sizes), weights=wts)
    for q in base:
        q.arrival = 0.0
    sat = summarize(Server(ex, int(0.8 * free), max_split=3).run(base))
    lam = rate_factor * sat["throughput_req_s"]
    reqs = synth.serving_stream(n_requests, rate=lam, sizes=tuple(sizes), weights=wts)
    run = summarize(Server(ex, int(0.8 * free), max_split=3).run(reqs))
    keep = ("requests", "ok", "failed", "p50_latency_s", "p99_latency_s", "mean_latency_s", "throughput_req_s",
            "voxel_cg_iters_per_s", "makespan_s", "failures", "split_increments")
    return {"workload": f"{n_requests} Poisson requests, Voronoi RVEs N in {sizes}, FP64/mixed 50/50, "
                        f"5-20 increments; classes per precision and size, continuous batching; an increment whose "
                        f"Newton iteration fails is halved, up to 3 times",
            "saturated": {k: sat[k] for k in keep},
            "poisson": dict({k: run[k] for k in keep}, rate_factor=rate_factor, rate_req_s=lam)}


if __name__ == "__main__":
    main()
