#!/usr/bin/env python3
"""Benchmark of the qHP TD-CFIE marching-on-in-time hot path on one MI355X.

Default workload: PEC sphere r = 1 m, icosphere level 4 (7680 edges),
c*dt = 0.02 m (K = 101 lags), one x-polarised wave along -z with a 150 MHz
modulated Gaussian pulse; synthetic, seeded, no dataset.

A step is one pass of the whole hot path: the history sum, the FP64 T_0
solve and the FP64 post-processing to the current j_i.  The FP64 assembly is
marched first with FP64 blocks (the plain FP64 path: LU back-solves, and the
inverse product), then in FP32 blocks (FP64 y and sums); a second assembly
keeps the raw lag matrices lag-banded and marches the factored history in
FP64 and with FP32 band values (the default headline, `value`).  Every form
is timed over --steps steps after --warmup, and marched again, untimed, over
a window that holds the pulse and its decay (600 steps; the pulse peaks near
step 145): `rel_err_vs_fp64` = max_i |j_i - j_i^FP64| / max_i |j_i^FP64| over
that window, against the FP64 LU march.  The default run adds the batched
form as `batched`: the 6000-edge torus with 128 waves, int8-digit blocks on
the int8 matrix cores against FP64, 300 steps.  Prints one JSON line.
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
BF16_MFMA_PEAK_TFLOPS = 2500.0
INT8_MFMA_PEAK_TOPS = 5000.0  # dense int8 matrix-core peak of the MI355X
FP64_MFMA_PEAK_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="sphere-large",
                    choices=["sphere-large", "sphere-small", "torus-batched", "uneven-batch", "warm-start",
                             "spectral"])
    ap.add_argument("--mesh", default="sphere", choices=["sphere", "torus"], help="warm-start mesh")
    ap.add_argument("--train-dirs", type=int, default=256, help="warm-start training directions")
    ap.add_argument("--train-steps", type=int, default=2000, help="warm-start training march length")
    ap.add_argument("--epochs", type=int, default=8, help="warm-start training passes")
    ap.add_argument("--eval-dirs", type=int, default=2, help="warm-start held-out directions")
    ap.add_argument("--scatterers", type=int, default=32, help="uneven-batch: march the first N of the 32")
    ap.add_argument("--precision", default=None,
                    choices=["f32", "f32a", "bf16", "bf16x2", "i8x4", "f64", "fac64", "fac32", "fp8"],
                    help="history form (default: fac32 = factored history, FP32 lag-banded raw matrices with FP64 "
                         "products and sums, for one wave; f32a = FP32 blocks with FP64 y and sums for "
                         "uneven-batch; i8x4 = int8 digit blocks on the int8 matrix cores for torus-batched)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a 4 GiB device copy first (reference for profiler byte counters)")
    ap.add_argument("--solver", default="inv", choices=["lu", "inv"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true", help="only the FP64 reference and the headline march")
    ap.add_argument("--err-steps", type=int, default=0,
                    help="steps of the untimed error marches (default: 600 for sphere-large, 300 for the torus)")
    ap.add_argument("--no-batched", action="store_true",
                    help="sphere-large: leave out the batched torus sub-record")
    ap.add_argument("--n-dirs", type=int, default=64, help="directions for torus-batched")
    a = ap.parse_args()
    if a.precision is None:
        a.precision = {"torus-batched": "i8x4", "sphere-large": "fac32", "sphere-small": "fac32"}.get(
            a.workload, "f32a")
    return a


def workload(name, n_dirs):
    from workloads import waves
    if name == "sphere-large":
        return waves.sphere_large()
    if name == "sphere-small":
        return waves.sphere_small()
    return waves.torus_batched(n_dirs)


def traffic_from_profile(kernel_name, variant=None):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel source and, for an autotuned kernel, on the
    variant in use (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        ent = rec.get("kernels", {}).get(kernel_name)
        if not ent:
            return None
        if variant is not None and ent.get("variant_index") is not None and ent["variant_index"] != variant:
            return None
        src = open(os.path.join(ROOT, "paper_2312_06367_amd", "csrc", ent["source"]), "rb").read()
        if ent.get("source_sha256") != hashlib.sha256(src).hexdigest():
            return None
        return ent["fetch_bytes_per_launch"] + ent["write_bytes_per_launch"]
    except Exception:
        return None


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return int(max([p.get("num_threads", 1) for p in threadpool_info() if p.get("user_api") == "blas"] or [1]))
    except Exception:
        return os.cpu_count() or 1


def oracle_step_seconds(ne, K, nrhs=1, budget_s=20.0):
    """Median seconds of one oracle marching step (history sum + LU solve) on
    host cores, from a bounded sample of the same shape: ks of the K lag
    blocks (random FP64 data, ne x ne, nrhs right-hand sides), the history
    time scaled to K lags.  Returns (seconds, ks, samples)."""
    import numpy as np
    import scipy.linalg as sla
    from oracle import mot
    rng = np.random.default_rng(0)
    ks = min(6, K)
    T = rng.standard_normal((ks + 1, ne, ne))
    T[0] += ne * np.eye(ne)
    ring = [rng.standard_normal((ne, nrhs)) if nrhs > 1 else rng.standard_normal(ne) for _ in range(ks)]
    lu = sla.lu_factor(T[0])
    r = rng.standard_normal((ne, nrhs)) if nrhs > 1 else rng.standard_normal(ne)
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
    return sorted(times)[len(times) // 2], ks, len(times)


def cpu_baseline(ne, K, budget_s=20.0):
    """The oracle's steps/s on the workload's shape (bounded sample)."""
    step_s, ks, n = oracle_step_seconds(ne, K, 1, budget_s)
    return {"value": 1.0 / step_s, "unit": "MOT steps/s", "cores": blas_threads(), "kind": "oracle",
            "sample": "oracle history sum over %d of the %d lag blocks (FP64 %dx%d, random data) + LU solve, "
                      "median of %d steps, history time scaled by %d/%d" % (ks, K, ne, ne, n, K, ks)}


def log(*x):
    print("[bench]", *x, file=sys.stderr, flush=True)


def bench_uneven(a):
    """32 seeded scatterers of uneven size (spheres, cubes, tori; 500-12000
    edges), 8 waves each, FP32 blocks (FP32 arithmetic, or FP64 y and sums
    with --precision f32a), marched together: one graph replay per step of
    grouped work-queue kernels."""
    import numpy as np
    import torch
    import paper_2312_06367_amd as qhp
    from workloads import waves
    cfgs = waves.uneven_batch()[: a.scatterers]
    n_total = cfgs[0].n_steps
    steps = min(a.steps, n_total - a.warmup)
    prec = a.precision if a.precision in ("f32", "f32a", "f64") else "f32"
    order = sorted(range(len(cfgs)), key=lambda i: -len(cfgs[i].mesh[1]))  # largest first: lowest memory peak
    solvers = [None] * len(cfgs)
    t0 = time.perf_counter()
    hist_bytes = 0
    work = []
    for i in order:
        c = cfgs[i]
        sv = qhp.Solver(c.dt, precision=prec, solver="inv")
        sv.mesh(*c.mesh)
        sv.assemble()
        sv.set_incident(c.waves, n_total)
        sv.release_assembly()
        inf = sv.info()
        solvers[i] = sv
        esz = {"f64": 8, "f32": 4, "f32a": 4}[prec]
        hist_bytes += inf["K"] * inf["ne"] * inf["ne"] * esz
        work.append((inf["ne"], inf["K"], i))
        log("scatterer %2d %-14s ne=%5d K=%3d slabs %.2f GB (%.0f s)" % (
            i, c.name, inf["ne"], inf["K"], inf["slab_bytes"] / 1e9, time.perf_counter() - t0))
    t_asm = time.perf_counter() - t0
    b = qhp.Batch(solvers)
    # outputs for the two smallest scatterers, checked against FP64 eager marches
    small = [w[2] for w in sorted(work)[:2]]
    nes = {w[2]: w[0] for w in work}
    jh = [None] * len(cfgs)
    for i in small:
        jh[i] = torch.zeros((n_total, nes[i], len(cfgs[i].waves)), dtype=torch.float64, device="cuda")
    b.run(a.warmup, [None if t is None else t[: a.warmup] for t in jh])
    torch.cuda.synchronize()
    tw = time.perf_counter()
    b.run(steps, [None if t is None else t[a.warmup: a.warmup + steps] for t in jh])
    torch.cuda.synchronize()
    wall = time.perf_counter() - tw
    ms = b.step_times(steps)
    p50, p99 = float(np.percentile(ms, 50)), float(np.percentile(ms, 99))
    log("batch: %d steps %.2f s, p50 %.3f ms, p99 %.3f ms" % (steps, wall, p50, p99))
    b.close()
    for sv in solvers:
        sv.close()
    torch.cuda.empty_cache()
    errs = {}
    for i in small:
        c = cfgs[i]
        sv = qhp.Solver(c.dt, precision="f64", solver="lu")
        sv.mesh(*c.mesh)
        sv.assemble()
        sv.set_incident(c.waves, n_total)
        ref = torch.zeros_like(jh[i])
        sv.run(a.warmup + steps, ref[: a.warmup + steps])
        sv.close()
        d = torch.linalg.vector_norm(jh[i][: a.warmup + steps] - ref[: a.warmup + steps], dim=1).max()
        errs[cfgs[i].name] = float(d / torch.linalg.vector_norm(ref, dim=1).max())
        log("scatterer %d (%s): current err vs FP64 eager %.2e" % (i, cfgs[i].name, errs[cfgs[i].name]))
    achieved = hist_bytes / (p50 * 1e-3) / 1e9
    out = {
        "metric": "MOT steps/s & history-sum HBM GB/s, batched FP32 vs plain FP64, rel err",
        "value": len(cfgs) * steps / wall,
        "unit": "scatterer MOT steps/s (%d scatterers per batch step)" % len(cfgs),
        "n_gpus": 1, "steps": steps, "warmup": a.warmup, "ms_per_step": 1e3 * wall / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": prec, "data": "synthetic",
        "config": {"workload": "uneven-batch-%d" % len(cfgs), "n_scatterers": len(cfgs), "n_rhs_each": 8, "c_dt_m": 0.05,
                   "ne": [cfgs[i].name for i in range(len(cfgs))], "slab_bytes_total": hist_bytes},
        "p50_step_ms": p50, "p99_step_ms": p99,
        "rel_err_vs_fp64": errs,
        "assembly_s": t_asm,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": None,
                     "kernel": "whole batch step (graph replay), lag-block bytes only",
                     "algorithmic_bytes_per_launch": hist_bytes, "kernel_ms_avg": p50},
    }
    if not a.no_cpu_baseline:
        sub = sorted(work)[:4] + sorted(work)[-1:]
        secs = [oracle_step_seconds(ne, K, 8, 8.0)[0] for ne, K, _ in sub]
        sub_work = sum(K * ne * ne for ne, K, _ in sub)
        all_work = sum(K * ne * ne for ne, K, _ in work)
        batch_s = sum(secs) * all_work / sub_work
        out["cpu_baseline"] = {
            "value": len(cfgs) / batch_s, "unit": out["unit"], "cores": blas_threads(), "kind": "oracle",
            "sample": "oracle steps (history over 6 lag blocks scaled to K, 8 right-hand sides, LU solve, random "
                      "FP64 data) of the 4 smallest and the largest scatterer, scaled to all 32 by K ne^2"}
    print(json.dumps(out), flush=True)


def bench_warm(a):
    """Learned warm start: train the perceptron on GPU marches of seeded
    directions, then march held-out directions with GMRES started cold, from
    y_{i-1}, by linear and quadratic extrapolation and by the network; LU and
    the explicit inverse beside them."""
    import numpy as np
    import torch
    import paper_2312_06367_amd as qhp
    from workloads import waves
    cfg = waves.sphere_large() if a.mesh == "sphere" else waves.torus_batched(1)
    xyz, tri = cfg.mesh
    w0 = cfg.waves[0]
    D = 2.0 if a.mesh == "sphere" else 2.6
    train = waves.batched_waves(a.train_dirs, 0, w0.f0, w0.bw, D, both_pols=False)
    held = waves.batched_waves(a.eval_dirs, 1, w0.f0, w0.bw, D, both_pols=False)
    # training marches: BF16-pair blocks on the matrix cores, all directions at once
    t0 = time.perf_counter()
    st = qhp.Solver(cfg.dt, precision="bf16x2", solver="inv")
    st.mesh(xyz, tri)
    st.assemble()
    inf = st.info()
    ne, K = inf["ne"], inf["K"]
    log("%s: ne=%d K=%d assembly (BF16 pairs) %.1f s" % (cfg.name, ne, K, time.perf_counter() - t0))
    n_tr = a.train_steps
    st.set_incident(train, n_tr)
    yh = torch.zeros((n_tr, ne, len(train)), dtype=torch.float64, device="cuda")
    t0 = time.perf_counter()
    for c0 in range(0, n_tr, 100):
        c1 = min(n_tr, c0 + 100)
        st.run(c1 - c0, None, yh[c0:c1])
        torch.cuda.synchronize()
        log("training marches: %d / %d steps (%.0f s)" % (c1, n_tr, time.perf_counter() - t0))
    t_data = time.perf_counter() - t0
    mt = qhp.MLP(st, hidden=256, seed=0)
    t0 = time.perf_counter()
    losses = []
    for e0 in range(0, a.epochs, 2):  # two passes per call, progress between calls
        losses += [float(v) for v in mt.train(yh, epochs=min(2, a.epochs - e0), batch=512, lr=1e-3, seed=e0)]
        log("training: %d / %d epochs (%.0f s), loss %s" % (len(losses), a.epochs, time.perf_counter() - t0,
                                                           " ".join("%.3e" % v for v in losses)))
    t_train = time.perf_counter() - t0
    params = mt.get_params()
    mt.close()
    st.close()
    del yh
    torch.cuda.empty_cache()
    # held-out marches: FP32 blocks with FP64 sums, one wave at a time
    t0 = time.perf_counter()
    sv = qhp.Solver(cfg.dt, precision="f32a", solver="inv")
    sv.mesh(xyz, tri)
    sv.assemble()
    log("assembly (FP32) %.1f s" % (time.perf_counter() - t0))
    m = qhp.MLP(sv, hidden=256, seed=0)
    m.set_params(params)
    sv.attach_mlp(m)
    n_ev = a.steps
    modes = {}

    def march(tag, setup):
        setup()
        tot_it, r0s, wall, net = 0, [], 0.0, 0
        for w in held:
            sv.gmres_reset()
            sv.set_incident([w], n_ev)
            torch.cuda.synchronize()
            tt = time.perf_counter()
            sv.run(n_ev)
            torch.cuda.synchronize()
            wall += time.perf_counter() - tt
            if tag.startswith("gmres"):
                st = sv.gmres_stats(n_ev)
                tot_it += st["iterations"]
                net += st["network_starts"]
                r0s.append(st["res0"][8:])
        rec = {"steps_per_s": len(held) * n_ev / wall}
        if r0s:
            r = np.concatenate(r0s)
            rec.update({"iterations_per_step": tot_it / (len(held) * n_ev),
                        "median_start_residual": float(np.median(r[r > 0])) if (r > 0).any() else 0.0})
            if tag == "gmres-best":
                rec["network_start_fraction"] = net / (len(held) * n_ev)
        modes[tag] = rec
        log("%-14s %s" % (tag, json.dumps(rec)))

    march("lu", lambda: sv.set_solver("lu"))
    march("inv", lambda: sv.set_solver("inv"))
    for warm in ("cold", "prev", "extrap", "quad", "mlp", "best"):
        march("gmres-" + warm, lambda warm=warm: sv.set_gmres(1e-10, 40, 4, warm))
    sv.attach_mlp(None)
    m.close()
    sv.close()
    head = modes["gmres-mlp"]
    out = {
        "metric": "MOT steps/s & history-sum HBM GB/s, batched FP32 vs plain FP64, rel err",
        "value": head["steps_per_s"], "unit": "MOT steps/s",
        "n_gpus": 1, "steps": n_ev, "warmup": 0, "ms_per_step": 1e3 / head["steps_per_s"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32-storage/f64-accumulate; perceptron bf16/f32", "data": "synthetic",
        "config": {"workload": "warm-start-" + cfg.name, "ne": ne, "K": K, "train_dirs": len(train),
                   "train_steps": n_tr, "epochs": a.epochs, "eval_dirs": len(held), "hidden": 256,
                   "gmres": {"tol": 1e-10, "m_max": 40, "max_refine": 4}},
        "modes": modes, "train_losses": losses, "training_data_s": t_data, "training_s": t_train,
    }
    print(json.dumps(out), flush=True)


def decay_radius(norms, start, window, floor=1e-200):
    """Late-time decay rate of a march whose excitation has passed: block
    maxima of |y_i| over windows from step start on (windows whose maximum
    fell below floor times the first are dropped), log-linear least squares,
    exp(slope).  The march applies the companion matrix once per step, so
    this is power iteration for its spectral radius."""
    import numpy as np
    for w in (window, window // 4, 2):  # shorter windows for marches that decay within a few of them
        nb = (len(norms) - start) // w
        m = np.array([norms[start + b * w:start + (b + 1) * w].max() for b in range(nb)])
        keep = (m > floor * m[0]) & (m > 1e-280)
        if keep.sum() >= 4:
            return float(np.exp(np.polyfit(np.arange(nb)[keep] * w, np.log(m[keep]), 1)[0]))
    return None


def bench_spectral(a):
    """cond_2(T_0) (power iteration), cond_1(T_0) and the companion spectral
    radius (from the late-time decay of an FP64 march) against mesh size and
    against the time step on the 480-edge sphere (the conditioning study of
    Sec. V-A, its ranges, and the small steps of the march workloads)."""
    import numpy as np
    import torch
    import paper_2312_06367_amd as qhp
    from workloads import meshes, waves

    f0 = waves.hz_to_per_m(50e6)

    def one(level, dt):
        xyz, tri = meshes.icosphere(level)
        t0 = time.perf_counter()
        s = qhp.Solver(dt, precision="f64", solver="inv")
        s.mesh(xyz, tri)
        s.assemble()
        inf = s.info()
        cond, cond2 = s.t0_condition(800)
        f = min(f0, 1.0 / (16.0 * dt))  # a pulse the time step resolves
        w = waves.Wave((0.0, 0.0, -1.0), (1.0, 0.0, 0.0), 1.0, waves.mod_gauss_t0(f, inf["diameter"]), 0, 0.0, f, f)
        # the fit starts once the pulse and two transits of the scatterer are over
        start = max(200, int(np.ceil((w.t0 + 8.0 / f + 2.0 * inf["diameter"]) / dt)))
        n = start + 800
        yh = torch.zeros((n, inf["ne"], 1), dtype=torch.float64, device="cuda")
        s.set_incident([w], n)
        s.run(n, None, yh)
        ny = torch.linalg.vector_norm(yh[:, :, 0], dim=1).cpu().numpy()
        s.close()
        del yh
        torch.cuda.empty_cache()
        rho = decay_radius(ny, start, 40)
        rec = {"ne": inf["ne"], "c_dt_m": dt, "K": inf["K"], "cond2_T0": cond2, "cond1_T0": cond, "companion_radius": rho,
               "steps": n, "fit_from_step": start, "seconds": time.perf_counter() - t0}
        log("ne=%5d c.dt=%9.4f K=%3d cond_2(T_0)=%8.4f cond_1(T_0)=%9.3f radius=%s (%d steps, %.1f s)"
            % (inf["ne"], dt, inf["K"], cond2, cond, "%.6f" % rho if rho is not None else "-", n, rec["seconds"]))
        return rec

    def safe(level, dt):
        try:
            return one(level, dt)
        except qhp.QhpError as e:  # recorded, not hidden
            log("ne level %d c.dt=%g: %s" % (level, dt, e))
            return {"level": level, "c_dt_m": dt, "error": str(e)}

    # the paper's two studies: mesh size at c dt = 1 m, time step on a 0.3 m mesh
    # from 0.25 m to 2048 m; and the same two at the small steps of the march
    # workloads (c dt = 0.05 m; 0.0125 m to 0.1 m)
    sweep_h = [safe(level, 1.0) for level in (1, 2, 3, 4)]
    sweep_dt = [safe(2, dt) for dt in (0.25, 1.0, 4.0, 16.0, 64.0, 256.0, 1024.0, 2048.0)]
    sweep_h_small = [safe(level, 0.05) for level in (1, 2, 3, 4)]
    sweep_dt_small = [safe(2, dt) for dt in (0.0125, 0.025, 0.05, 0.1)]
    ok = [r for r in sweep_h + sweep_dt if "cond2_T0" in r]
    out = {"metric": "cond_2(T_0) and companion spectral radius vs mesh size and time step",
           "value": max(r["cond2_T0"] for r in ok) if ok else None,
           "unit": "largest cond_2(T_0) over the mesh-size and time-step sweeps",
           "n_gpus": 1, "higher_is_better": False, "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "spectral", "mesh": "icospheres, radius 1 m", "wave": "modulated Gaussian, 50 MHz"},
           "sweep_h": sweep_h, "sweep_dt": sweep_dt, "sweep_h_small_dt": sweep_h_small,
           "sweep_dt_small": sweep_dt_small}
    print(json.dumps(out), flush=True)


DENSE_ESZ = {"f64": 8, "f32": 4, "f32a": 4, "bf16": 2, "bf16x2": 4, "i8x4": 4, "fp8": 4}
DTYPE = {"f32": "f32", "bf16": "bf16-storage/f32", "f32a": "f32-storage/f64-accumulate", "f64": "f64",
         "bf16x2": "bf16-pair-storage/bf16-mfma/f32-accumulate",
         "i8x4": "int8-digit-storage/int8-mfma/exact-int32-per-lag/f64-across-lags",
         "fac64": "f64 (factored, lag-banded)", "fac32": "f32-band-storage/f64-products-and-sums (factored)",
         "fp8": "fp8-e4m3-values-in-f32-words/f64-accumulate (accuracy study)"}


def bench_single(a, cfg, precision, steps, warmup, err_steps, quick, with_cpu):
    """One workload marched in the requested form and beside it the plain
    FP64 path (LU and inverse) and the other forms (unless quick).  Timed
    marches: warmup + steps from the start of the excitation.  Errors: every
    form marched again for err_steps steps (untimed), max over steps of
    |j_i - j_i^FP64| / max_i |j_i^FP64|."""
    import torch
    import paper_2312_06367_amd as qhp
    xyz, tri = cfg.mesh
    n_rhs = len(cfg.waves)
    n_total = warmup + steps
    t0 = time.perf_counter()
    s = qhp.Solver(cfg.dt, precision="f64", solver="lu")
    s.mesh(xyz, tri)
    s.assemble()
    torch.cuda.synchronize()
    t_asm = time.perf_counter() - t0
    inf = s.info()
    ne, K = inf["ne"], inf["K"]
    raw_nnz = inf["raw_nnz"]
    peak_step = int(max(w.t0 for w in cfg.waves) / cfg.dt)
    n_err = max(err_steps, n_total)
    log("%s: ne=%d K=%d n_rhs=%d assembly %.1f s; pulse peak near step %d, errors over %d steps"
        % (cfg.name, ne, K, n_rhs, t_asm, peak_step, n_err))

    def march(tag, solver, sv):
        sv.set_solver(solver)
        sv.set_incident(cfg.waves, n_total)
        jh = torch.zeros((n_total, ne, n_rhs), dtype=torch.float64, device="cuda")
        sv.run(warmup, jh[:warmup])
        torch.cuda.synchronize()
        sv.profile(True)
        torch.cuda.synchronize()
        tw0 = time.perf_counter()
        sv.run(steps, jh[warmup:])
        torch.cuda.synchronize()
        wall = time.perf_counter() - tw0
        ms_hist, launches = sv.hist_time()
        band = sv.band_time()
        sv.profile(False)
        hist = ms_hist / max(launches, 1)
        info = sv.info()
        log("%-9s %-3s: %d steps %.3f s = %.1f steps/s; history %.3f ms (variant %d, %d splits)"
            % (tag, solver, steps, wall, steps / wall, hist, info["hist_variant"], info["hist_splits"]))
        rec = {"steps_per_s": steps / wall, "wall": wall, "hist_ms": hist, "variant": info["hist_variant"],
               "info": info}
        if band[2] > 0:
            rec["band_ms"] = (band[0] / band[2], band[1] / band[2])
            log("%-9s %-3s: far-lag passes (one per %d steps) %.3f ms (edge pairs) + %.3f ms (triangle pairs)"
                % (tag, solver, info["band_block"], rec["band_ms"][0], rec["band_ms"][1]))
        return rec

    def err_march(sv):
        sv.set_incident(cfg.waves, n_err)
        jh = torch.zeros((n_err, ne, n_rhs), dtype=torch.float64, device="cuda")
        for c0 in range(0, n_err, 500):  # progress between chunks
            sv.run(min(500, n_err - c0), jh[c0:c0 + 500])
            torch.cuda.synchronize()
        return jh

    ref = {}

    def rel(jx):
        jr = ref["j"]
        d = torch.linalg.vector_norm(jx - jr, dim=1).max().item()
        return d / torch.linalg.vector_norm(jr, dim=1).max().item()

    runs = {}
    diverged = {}
    other = {"lu": "inv", "inv": "lu"}[a.solver]
    runs["f64_lu"] = march("f64", "lu", s)
    ref["j"] = err_march(s)
    runs["f64_lu"]["err"] = 0.0
    if not quick or a.solver == "inv":
        runs["f64_inv"] = march("f64", "inv", s)
        runs["f64_inv"]["err"] = rel(err_march(s))
    fac = precision.startswith("fac")
    dense_forms = [] if (fac and quick) else ([precision] if not fac else ["f32a"])
    if precision == "f64":
        dense_forms = []
    for p in dense_forms:
        s.set_precision(p)
        for sol in ([a.solver] if quick else [a.solver, other]):
            key = "%s_%s" % (p, sol)
            try:
                runs[key] = march(p, sol, s)
                runs[key]["err"] = rel(err_march(s))
            except qhp.QhpError as e:  # a form that does not stay finite on this workload
                log("%-9s %-3s: %s" % (p, sol, e))
                runs.pop(key, None)
                diverged[p] = str(e)
                break
        if not quick and p in ("f32", "f32a"):
            twin = "f32" if p == "f32a" else "f32a"
            s.set_precision(twin)
            key = "%s_%s" % (twin, a.solver)
            runs[key] = march(twin, a.solver, s)
            runs[key]["err"] = rel(err_march(s))
    if not quick and n_rhs > 1:  # the other multi-right-hand-side forms, each assembled in its own storage
        for p in ("f32", "bf16", "bf16x2", "i8x4"):
            if p == precision:
                continue
            sv = qhp.Solver(cfg.dt, precision=p, solver=a.solver)
            sv.mesh(xyz, tri)
            sv.assemble()
            key = "%s_%s" % (p, a.solver)
            try:
                runs[key] = march(p, a.solver, sv)
                runs[key]["err"] = rel(err_march(sv))
            except qhp.QhpError as e:  # a form that does not stay finite on this workload
                log("%-9s %-3s: %s" % (p, a.solver, e))
                runs.pop(key, None)
                diverged[p] = str(e)
            sv.close()
    s.close()
    torch.cuda.empty_cache()
    if fac:  # the factored forms: their own assembly (raw lag matrices, bands)
        t0 = time.perf_counter()
        sf = qhp.Solver(cfg.dt, precision="fac64", solver=a.solver)
        sf.mesh(xyz, tri)
        sf.assemble()
        torch.cuda.synchronize()
        log("factored assembly %.1f s" % (time.perf_counter() - t0))
        for p in (["fac64", "fac32"] if precision == "fac32" else ["fac64"]) if not quick else [precision]:
            if p != sf.precision:
                sf.set_precision(p)
            key = "%s_%s" % (p, a.solver)
            runs[key] = march(p, a.solver, sf)
            runs[key]["err"] = rel(err_march(sf))
        sf.close()
        torch.cuda.empty_cache()
    key = "%s_%s" % (precision, a.solver) if precision != "f64" else "f64_" + a.solver
    if key not in runs:  # the requested form diverged: reported, no throughput
        return {"metric": "MOT steps/s & history-sum HBM GB/s, batched FP32 vs plain FP64, rel err", "value": None,
                "unit": "MOT steps/s", "n_gpus": 1, "steps": steps, "warmup": warmup, "higher_is_better": True,
                "vs_baseline": None, "dtype": DTYPE[precision], "data": "synthetic",
                "config": {"workload": cfg.name, "ne": ne, "K": K, "c_dt_m": cfg.dt, "n_rhs": n_rhs,
                           "history": precision}, "diverged": diverged.get(precision, "not marched"),
                "fp64_steps_per_s": runs["f64_lu"]["steps_per_s"]}
    head = runs[key]
    hinf = head["info"]
    flops_per_launch = 2.0 * K * ne * ne * n_rhs
    ysz = 8 if precision in ("f64", "f32a", "fp8") else 4
    bytes_per_launch = K * ne * ne * DENSE_ESZ.get(precision, 8) + K * ne * n_rhs * ysz
    if fac:
        # the dominant kernel: the banded product over the edge pairs
        fp32 = precision == "fac32"
        # the far lags' pass over the edge pairs (once per band_block steps)
        kname = "k_band<%s, %d, %d, %d>" % ("float" if fp32 else "double", hinf["band_waves_pairs"],
                                             hinf["band_pieces_pairs"], hinf["band_block"])
        kb = hinf["band_bytes_pairs"]
        achieved = kb / (head["band_ms"][0] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic_from_profile(kname),
                "kernel": kname, "algorithmic_bytes_per_launch": kb, "kernel_ms_avg": head["band_ms"][0],
                "values_per_launch": hinf["band_nnz_pairs"],
                "steps_per_pass": hinf["band_block"],
                # one pass serves band_block steps: band_block FP64 products per value
                "fp64_tflops": 2.0 * hinf["band_nnz_pairs"] * max(hinf["band_block"], 1)
                / (head["band_ms"][0] * 1e-3) / 1e12,
                "fp64_peak_tflops": 78.6,
                "band_bytes_per_step": kb / max(hinf["band_block"], 1) + hinf["band_bytes_near_pairs"],
                "triangle_pair_band": {"kernel": "k_band<%s, %d, %d, %d>" % ("float" if fp32 else "double",
                                                                              hinf["band_waves_cells"],
                                                                              hinf["band_pieces_cells"],
                                                                              hinf["band_block"]),
                                       "bytes": hinf["band_bytes_cells"], "ms_avg": head["band_ms"][1],
                                       "gbps": hinf["band_bytes_cells"] / (head["band_ms"][1] * 1e-3) / 1e9}}
    elif n_rhs == 1:
        kname = {"f64": "k_hist_gemv<double,double,double>", "f32": "k_hist_gemv<float,float,float>",
                 "f32a": "k_hist_gemv<float,double,double>", "fp8": "k_hist_gemv<float,double,double>",
                 "bf16": "k_hist_gemv<unsigned short,float,float>"}[precision]
        achieved = bytes_per_launch / (head["hist_ms"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic_from_profile(kname, head["variant"]),
                "kernel": kname, "variant": head["variant"], "algorithmic_bytes_per_launch": bytes_per_launch,
                "kernel_ms_avg": head["hist_ms"]}
    elif precision in ("bf16", "bf16x2"):
        # BF16 matrix cores: five (pair) or two BF16 products per term; the
        # streamed block bytes bound the kernel
        kname = "k_hist_mfma<%s>" % ("true" if precision == "bf16x2" else "false")
        achieved = bytes_per_launch / (head["hist_ms"] * 1e-3) / 1e9
        products = 5 if precision == "bf16x2" else 2
        executed = products * flops_per_launch / (head["hist_ms"] * 1e-3) / 1e12
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic_from_profile(kname),
                "kernel": kname, "algorithmic_bytes_per_launch": bytes_per_launch,
                "kernel_ms_avg": head["hist_ms"],
                "bf16_mfma_executed_tflops": executed, "bf16_mfma_frac": executed / BF16_MFMA_PEAK_TFLOPS}
    elif precision == "i8x4":
        # int8 matrix cores: 13 digit products per term, exact int32 sums per lag;
        # the kernel is the autotuned variant (the library's variant table, in order)
        kname = ["k_hist_i8<2,2,4,2,2>", "k_hist_i8d<2,2,4,2,2>", "k_hist_i8d<2,2,4,2,3>"][head["variant"]]
        ops = 13 * flops_per_launch
        achieved = ops / (head["hist_ms"] * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": INT8_MFMA_PEAK_TOPS, "unit": "TOP/s",
                "frac": achieved / INT8_MFMA_PEAK_TOPS, "traffic": traffic_from_profile(kname),
                "kernel": kname, "algorithmic_int8_ops_per_launch": ops,
                "kernel_ms_avg": head["hist_ms"],
                "hbm_gbps": bytes_per_launch / (head["hist_ms"] * 1e-3) / 1e9}
    else:
        kname = "k_hist_gemm<float>" if precision == "f32" else "k_hist_gemm<double>"
        peak = FP32_MFMA_PEAK_TFLOPS if precision == "f32" else FP64_MFMA_PEAK_TFLOPS
        achieved = flops_per_launch / (head["hist_ms"] * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": traffic_from_profile(kname),
                "kernel": kname, "algorithmic_flops_per_launch": flops_per_launch,
                "kernel_ms_avg": head["hist_ms"]}

    def hist_gbps(key, rr):
        p = key.split("_")[0]
        if p.startswith("fac"):
            return rr["info"]["slab_bytes"] / (rr["hist_ms"] * 1e-3) / 1e9
        ys = 8 if p in ("f64", "f32a", "fp8") else 4
        return (K * ne * ne * DENSE_ESZ[p] + K * ne * n_rhs * ys) / (rr["hist_ms"] * 1e-3) / 1e9

    forms = {}
    for key, rr in runs.items():
        forms[key] = {"steps_per_s": rr["steps_per_s"], "history_ms": rr["hist_ms"],
                      "history_gbps": hist_gbps(key, rr), "rel_err_vs_fp64_lu": rr["err"],
                      "history_bytes": rr["info"]["slab_bytes"]}
        if "band_ms" in rr:
            forms[key]["band_ms"] = list(rr["band_ms"])
    for p, msg in diverged.items():
        forms["%s_%s" % (p, a.solver)] = {"diverged": msg}
    out = {
        "metric": "MOT steps/s & history-sum HBM GB/s, batched FP32 vs plain FP64, rel err",
        "value": head["steps_per_s"],
        "unit": "MOT steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": 1e3 * head["wall"] / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[precision],
        "data": "synthetic",
        "config": {"workload": cfg.name, "ne": ne, "K": K, "c_dt_m": cfg.dt, "n_rhs": n_rhs,
                   "history": precision, "solve": "fp64-" + a.solver, "post_processing": "fp64"},
        "history_gbps": hist_gbps(key, head),
        "rel_err_vs_fp64": head["err"],
        "rel_err_steps": n_err,
        "pulse_peak_step": peak_step,
        "fp64_steps_per_s": runs["f64_lu"]["steps_per_s"],
        "fp64_inv_steps_per_s": runs["f64_inv"]["steps_per_s"] if "f64_inv" in runs else None,
        "forms": forms,
        "assembly_s": t_asm,
        "roofline": roof,
        "raw_nnz": raw_nnz,
        "dense_slab_bytes_fp32": K * ne * ne * 4,
    }
    if with_cpu:
        out["cpu_baseline"] = cpu_baseline(ne, K)
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: the marching solver runs on a single MI355X "
              "(--gpus %d is not supported)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    torch.cuda.set_device(0)
    if a.workload == "uneven-batch":
        return bench_uneven(a)
    if a.workload == "warm-start":
        return bench_warm(a)
    if a.workload == "spectral":
        return bench_spectral(a)
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
    cfg = workload(a.workload, a.n_dirs)
    err_steps = a.err_steps if a.err_steps else {"sphere-large": 600, "torus-batched": 300}.get(a.workload, 400)
    out = bench_single(a, cfg, a.precision, a.steps, a.warmup, err_steps, a.quick, not a.no_cpu_baseline)
    if a.workload == "sphere-large" and not a.no_batched:
        # the batched form: torus 6000 edges x 128 waves, int8 digits against FP64
        tor = workload("torus-batched", 64)
        sub = bench_single(a, tor, "i8x4", min(a.steps, 300), min(a.warmup, 20), 300, True, False)
        out["batched"] = {k: sub[k] for k in ("value", "unit", "steps", "warmup", "ms_per_step", "dtype", "config",
                                              "history_gbps", "rel_err_vs_fp64", "rel_err_steps",
                                              "pulse_peak_step", "fp64_steps_per_s", "fp64_inv_steps_per_s",
                                              "forms", "roofline")}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
