#!/usr/bin/env python3
"""Benchmark of the qHP TD-CFIE marching-on-in-time hot path on one MI355X.

Default workload: PEC sphere r = 1 m, icosphere level 4 (7680 edges),
c*dt = 0.02 m (K = 101 lag blocks), one x-polarised wave along -z with a
150 MHz modulated Gaussian pulse; synthetic, seeded, no dataset.

A step is one pass of the whole hot path: the history sum over T_1..T_K, the
FP64 T_0 solve and the FP64 post-processing to the current j_i.  The FP64
assembly is marched first with FP64 slabs (the plain FP64 path, LU
back-solves and the inverse product), then re-stored in the requested
precision (default FP32) and marched again; `value` is the steps/s of that
march, `rel_err_vs_fp64` = max_i |j_i - j_i^{FP64}| / max_i |j_i^{FP64}|.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="sphere-large", choices=["sphere-large", "sphere-small", "torus-batched"])
    ap.add_argument("--precision", default="f32a", choices=["f32", "f32a", "bf16", "f64"],
                    help="slab storage / history arithmetic: f32a = FP32 blocks with FP64 y and sums")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a 4 GiB device copy first (reference for profiler byte counters)")
    ap.add_argument("--solver", default="inv", choices=["lu", "inv"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true", help="only the FP64 reference and the headline march")
    ap.add_argument("--n-dirs", type=int, default=64, help="directions for torus-batched")
    return ap.parse_args()


def workload(name, n_dirs):
    from workloads import waves
    if name == "sphere-large":
        return waves.sphere_large()
    if name == "sphere-small":
        return waves.sphere_small()
    return waves.torus_batched(n_dirs)


def traffic_from_profile(kernel_name):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        src = open(os.path.join(ROOT, "paper_2312_06367_amd", "csrc", "march.hip"), "rb").read()
        if rec.get("source_sha256") != hashlib.sha256(src).hexdigest():
            return None
        ent = rec.get("kernels", {}).get(kernel_name)
        return None if not ent else ent["fetch_bytes_per_launch"] + ent["write_bytes_per_launch"]
    except Exception:
        return None


def cpu_baseline(ne, K, budget_s=20.0):
    """Oracle marching step (history sum + LU solve) on host cores, on a
    bounded sample of the same shape: ks of the K lag blocks (random FP64
    data, ne x ne), the history time scaled to K lags."""
    import numpy as np
    import scipy.linalg as sla
    from oracle import mot
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info() if p.get("user_api") == "blas"] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    rng = np.random.default_rng(0)
    ks = 6
    T = rng.standard_normal((ks + 1, ne, ne))
    T[0] += ne * np.eye(ne)
    ring = [rng.standard_normal(ne) for _ in range(ks)]
    lu = sla.lu_factor(T[0])
    r = rng.standard_normal(ne)
    times = []
    t_end = time.perf_counter() + budget_s
    for _ in range(6):
        t0 = time.perf_counter()
        h = mot.history_sum(T, ring, ks + 1)
        t1 = time.perf_counter()
        sla.lu_solve(lu, r - h)
        t2 = time.perf_counter()
        times.append(((t1 - t0) * K / ks) + (t2 - t1))
        if time.perf_counter() > t_end:
            break
    step_s = sorted(times)[len(times) // 2]
    return {"value": 1.0 / step_s, "unit": "MOT steps/s", "cores": int(threads), "kind": "oracle",
            "sample": "oracle history sum over %d of the %d lag blocks (FP64 %dx%d, random data) + LU solve, "
                      "median of %d steps, history time scaled by %d/%d" % (ks, K, ne, ne, len(times), K, ks)}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: this build runs the marching solver on a single MI355X "
              "(--gpus %d is not supported)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2312_06367_amd as qhp

    torch.cuda.set_device(0)
    cfg = workload(a.workload, a.n_dirs)
    xyz, tri = cfg.mesh
    n_rhs = len(cfg.waves)
    n_total = a.warmup + a.steps
    t0 = time.perf_counter()
    s = qhp.Solver(cfg.dt, precision="f64", solver="lu")
    s.mesh(xyz, tri)
    s.assemble()
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - t0
    inf = s.info()
    ne, K = inf["ne"], inf["K"]
    log = lambda *x: print("[bench]", *x, file=sys.stderr, flush=True)
    log("%s: ne=%d K=%d n_rhs=%d assembly %.1f s" % (cfg.name, ne, K, n_rhs, t_asm))

    def march(tag, solver):
        s.set_solver(solver)
        s.set_incident(cfg.waves, n_total)
        jh = torch.zeros((n_total, ne, n_rhs), dtype=torch.float64, device="cuda")
        s.run(a.warmup, jh[: a.warmup])
        torch.cuda.synchronize()
        s.profile(True)
        torch.cuda.synchronize()
        tw0 = time.perf_counter()
        s.run(a.steps, jh[a.warmup:])
        torch.cuda.synchronize()
        wall = time.perf_counter() - tw0
        ms_hist, launches = s.hist_time()
        s.profile(False)
        hist = ms_hist / max(launches, 1)
        log("%-9s %-3s: %d steps %.3f s = %.1f steps/s; history kernel %.3f ms (variant %d, %d splits)"
            % (tag, solver, a.steps, wall, a.steps / wall, hist, s.info()["hist_variant"], s.info()["hist_splits"]))
        return {"j": jh, "steps_per_s": a.steps / wall, "wall": wall, "hist_ms": hist}

    def rel(jx, jref):
        d = torch.linalg.vector_norm(jx - jref, dim=1).max().item()
        return d / torch.linalg.vector_norm(jref, dim=1).max().item()

    def gbps(prec, hist_ms):
        esz = {"f64": 8, "f32": 4, "f32a": 4, "bf16": 2}[prec]
        ysz = 8 if prec in ("f64", "f32a") else 4
        return (K * ne * ne * esz + K * ne * n_rhs * ysz) / (hist_ms * 1e-3) / 1e9

    if a.calibrate_copy:
        # plain device copy of known size, for scaling HBM counters of the profiler
        nbytes = 1 << 32
        src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d bytes read, %d bytes written" % (nbytes, nbytes))
        del src, dst
        torch.cuda.empty_cache()

    runs = {}
    other = {"lu": "inv", "inv": "lu"}[a.solver]
    runs["f64_lu"] = march("f64", "lu")
    if not a.quick or a.solver == "inv":
        runs["f64_inv"] = march("f64", "inv")
    if a.precision != "f64":
        s.set_precision(a.precision)
        runs["head"] = march(a.precision, a.solver)
        runs["%s_%s" % (a.precision, a.solver)] = runs["head"]
        if not a.quick:
            runs["%s_%s" % (a.precision, other)] = march(a.precision, other)
            if a.precision in ("f32", "f32a"):
                twin = "f32" if a.precision == "f32a" else "f32a"
                s.set_precision(twin)
                runs["%s_%s" % (twin, a.solver)] = march(twin, a.solver)
    else:
        runs["head"] = runs["f64_" + a.solver]
    head = runs["head"]
    jref = runs["f64_lu"]["j"]
    esz = {"f64": 8, "f32": 4, "f32a": 4, "bf16": 2}[a.precision]
    ysz = 8 if a.precision in ("f64", "f32a") else 4
    bytes_per_launch = K * ne * ne * esz + K * ne * n_rhs * ysz
    flops_per_launch = 2.0 * K * ne * ne * n_rhs
    if n_rhs == 1:
        kname = {"f64": "k_hist_gemv<double,double,double>", "f32": "k_hist_gemv<float,float,float>",
                 "f32a": "k_hist_gemv<float,double,double>", "bf16": "k_hist_gemv<unsigned short,float,float>"}[a.precision]
        achieved = bytes_per_launch / (head["hist_ms"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic_from_profile(kname),
                "kernel": kname, "algorithmic_bytes_per_launch": bytes_per_launch,
                "kernel_ms_avg": head["hist_ms"]}
    else:
        kname = "k_hist_gemm<%s>" % ("unsigned short" if a.precision == "bf16" else "float")
        achieved = flops_per_launch / (head["hist_ms"] * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP32_MFMA_PEAK_TFLOPS, "traffic": traffic_from_profile(kname),
                "kernel": kname, "algorithmic_flops_per_launch": flops_per_launch,
                "kernel_ms_avg": head["hist_ms"]}
    forms = {}
    for key, rr in runs.items():
        if key == "head" or key in forms:
            continue
        prec = key.split("_")[0]
        forms[key] = {"steps_per_s": rr["steps_per_s"], "history_ms": rr["hist_ms"],
                      "history_gbps": gbps(prec, rr["hist_ms"]), "rel_err_vs_fp64_lu": rel(rr["j"], jref)}
    out = {
        "metric": "MOT steps/s & history-sum HBM GB/s, batched FP32 vs plain FP64, rel err",
        "value": head["steps_per_s"],
        "unit": "MOT steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * head["wall"] / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "bf16": "bf16-storage/f32", "f32a": "f32-storage/f64-accumulate", "f64": "f64"}[a.precision],
        "data": "synthetic",
        "config": {"workload": cfg.name, "ne": ne, "K": K, "c_dt_m": cfg.dt, "n_rhs": n_rhs,
                   "slab_storage": a.precision, "solve": "fp64-" + a.solver, "post_processing": "fp64"},
        "history_gbps": gbps(a.precision, head["hist_ms"]),
        "rel_err_vs_fp64": rel(head["j"], jref),
        "fp64_steps_per_s": runs["f64_lu"]["steps_per_s"],
        "forms": forms,
        "assembly_s": t_asm,
        "roofline": roof,
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(ne, K)
    s.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
