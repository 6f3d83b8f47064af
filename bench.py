"""Benchmark of the projection hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload mixed_channel] [--precision mixed]

A step is one full projection (immersed-body forcing -> Poisson right-hand side -> Poisson
solve from a zero guess to relative residual 1e-10 -> velocity correction) on the 32x16x16
cube channel with a sphere (33.6M cells, 16^3 cells per cube), inputs resident in HBM.
Prints one JSON line:
  value        Poisson cell-updates per second (fine-level cells x fine-level stencil
               applications per step: smoothing sweeps, residuals and operator applies)
  roofline     the dominant kernel's algorithmic bytes per launch / its mean launch time,
               timed with HIP events on the launch stream over the timed steps, against 8 TB/s
  fp64_*       the same step solved all in FP64 (time-to-tolerance comparison)
  cpu_baseline the FP64 CPU oracle on this host (7-point operator throughput, single thread)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0

# Algorithmic bytes per fine-level cell of one launch (halo / face traffic excluded), by
# timer class, for inner precision size s (4 for mixed, 8 for fp64) and field size f.
def alg_bytes_per_cell(cls, s, f, body=1.0):
    """Algorithmic bytes per cell of the class's level (face buffers excluded), or None for
    classes that are not a streaming pass (the cube-graph solve, the scalar finalize).
    s, f: bytes per solver value and per field value; body: the fraction of cubes that hold
    some nonzero volume fraction (the only ones the 16^3 forcing kernel reads and stores)."""
    return {
        "presmooth16": 2 * s + s / 8,    # read b; write x and the restricted residual
        "preupd16": 4 * s + s / 8,       # the same with the previous step's r update fused in:
                                         # read r, q; write r, x and the restricted residual
        "presmooth8": 3 * s + s / 8,     # below the finest level b is completed (its cross-cube
        "presmooth4": 3 * s + s / 8,     # terms) and written back as well
        "presmooth2": 3 * s + s / 8,
        "postsmooth16": 4 * s + s / 8,   # read x, b, q, coarse correction; write x
        "postsmooth8": 3 * s + s / 8,    # read x, b, coarse correction; write x
        "postsmooth4": 3 * s + s / 8,
        "postsmooth2": 3 * s + s / 8,
        "restrict2": s / 4,              # the one-cell-per-cube residual's cross-cube terms
        "apply16": 4 * s,                # read z, p; write p, q
        "update": 3 * s,                 # read r, q; write r
        "rprobe": 2 * s,                 # read r, q (<r - alpha q, r - alpha q> only)
        "xupdate": 3 * s,                # read x, p; write x (beside the next V-cycle)
        "resid64": 16 + s,               # read p, b (FP64); write r
        "ir": 8 + 2 * s + 8,             # read p, d and the inner solve's last direction; write p
        "force": f + 6 * f * body,       # read alpha; in body cubes read u~ (3), write u* (3)
        "div": 3 * f + 8,                # read u* (3); write b
        "correct": 8 + 6 * f,            # read p, u* (3); write u_new (3)
    }.get(cls)


def level_cells(cls, n_cells, n):
    """Cells of the per-cube level a class runs on (the trailing edge length in its name)."""
    digits = "".join(ch for ch in cls if ch.isdigit())
    if cls in ("resid64",) or not digits:
        return n_cells
    return n_cells * (int(digits) / n) ** 3


CLASSES = ("presmooth16", "preupd16", "postsmooth16", "apply16", "update", "rprobe", "xupdate", "resid64", "ir",
           "coarse", "force", "div", "correct", "presmooth8", "postsmooth8", "presmooth4",
           "postsmooth4", "presmooth2", "postsmooth2", "restrict2", "finalize")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_hash():
    """sha256 of the library sources: counter figures recorded for other sources are stale."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1808_04099_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()


def measured_traffic(kernel_cls, workload_name, precision):
    """HBM bytes per launch of a kernel class from the recorded rocprofv3 FETCH_SIZE and
    WRITE_SIZE passes (scaled by the copy-kernel calibration), or None when no figure exists
    for these sources."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_sha256") != source_hash():
        return None
    e = d.get("kernels", {}).get(f"{workload_name}/{precision}/{kernel_cls}")
    return None if e is None else e.get("hbm_bytes_per_launch")


def copy_probe(nbytes=1 << 30, reps=10):
    """Device-to-device copy of nbytes (read + write) with torch: the practical HBM ceiling,
    and the known-size kernel that calibrates the byte counters."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes_per_copy": 2 * nbytes, "ms": ms, "gbs": 2 * nbytes / (ms * 1e-3) / 1e9}


def workload(name):
    from bcm_inputs import configs
    if name == "mixed_channel":
        return configs.mixed_channel(), ("mixed_channel: 32x16x16 cubes of 16^3 (33,554,432 "
                                         "cells) on [0,2]x[0,1]^2, inflow/outflow/slip, sphere "
                                         "r=0.15 as volume fraction, 32-mode smooth field + U_in=1")
    if name == "sphere_channel":
        return configs.sphere_channel(), ("sphere_channel: 16x8x8 cubes of 16^3 (4,194,304 "
                                          "cells), sphere r=0.15, u=(1,0,0)+0.05U[-1,1]")
    if name == "small_box":
        return configs.small_box(), "small_box: 4x4x4 cubes of 16^3, open box"
    if name == "multilevel":
        pr = configs.multilevel()
        m = pr["mesh"]
        return pr, (f"multilevel: {m.n_cubes} cubes of 16^3 ({m.n_cells:,} cells) at levels 0-2 "
                    f"(2:1 faces) on [0,2]x[0,1]^2, inflow/outflow/slip, box + ellipsoid body as "
                    f"volume fraction, u=(1,0,0)+0.05U[-1,1]")
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(pr, seconds=10.0):
    """The oracle timed on this host.  Uniform meshes: its 7-point operator on the global array
    (NumPy, one thread) applied to the full field for ~seconds, plus one full oracle projection
    (spectral solve, all cores).  Multi-level meshes: its cell-by-cell operator (pure Python,
    one thread) on seeded random cells for ~seconds."""
    import numpy as np
    m = pr["mesh"]
    if len(set(m.level.tolist())) > 1:
        from oracle.sample import CellSampler
        cs = CellSampler(m)
        p = np.random.default_rng(0).standard_normal(m.n_cells)
        cells = np.random.default_rng(1).integers(0, m.n_cells, 1 << 20)
        t0 = time.perf_counter()
        done = 0
        while time.perf_counter() - t0 < seconds and done < cells.size:
            cs.laplacian(p, int(cells[done]))
            done += 1
        dt = time.perf_counter() - t0
        return dict(value=done / dt, unit="cell-updates/s", cores=1, kind="oracle",
                    sample=(f"{done} seeded random cells of the {m.n_cells}-cell multi-level "
                            f"mesh, each one application of the oracle's cell-by-cell FP64 "
                            f"finite-volume operator (pure Python, single thread)"),
                    oracle_projection_s=None)
    from oracle import UniformGrid
    ug = UniformGrid(m)
    g = ug.to_global(np.random.default_rng(0).standard_normal(m.n_cells))
    t0 = time.perf_counter()
    reps = 0
    while True:
        ug.laplacian(g)
        reps += 1
        if time.perf_counter() - t0 >= seconds:
            break
    t_apply = (time.perf_counter() - t0) / reps
    t1 = time.perf_counter()
    ug.project(pr["u"], pr["alpha"], (0.0, 0.0, 0.0), pr["U_in"], pr["dt"], pr["rho"])
    t_proj = time.perf_counter() - t1
    return dict(value=m.n_cells / t_apply, unit="cell-updates/s", cores=1,
                kind="oracle",
                sample=(f"{reps} applications of the oracle's FP64 7-point operator (array form, "
                        f"NumPy, single thread) to the full {m.n_cells}-cell field; "
                        f"the oracle's full projection step (exact DCT solve, scipy.fft on "
                        f"{os.cpu_count()} threads) took {t_proj:.2f} s"),
                oracle_projection_s=t_proj)


def next_rows(pr, mesh, args):
    """The momentum sub-step, the Lagrangian-particle forcing and the checkpoint codec on the
    same mesh (FP64 fields), each timed with HIP events on the library's stream (timer classes
    'momentum', 'ib', 'codec') over args.steps calls after one warm-up call."""
    import numpy as np
    import torch
    from bcm_inputs import sphere_particles
    from paper_1808_04099_amd import Plan
    m = pr["mesh"]
    n_cells = m.n_cells
    plan = Plan(mesh, precision="fp64")
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a).reshape(-1)).to("cuda")
    u = [dev(pr["u"][d]) for d in range(3)]
    out = {}

    def timed(cls, fn):
        fn()
        torch.cuda.synchronize()
        plan.timing_enable(cls)
        t0 = time.perf_counter()
        res = [fn() for _ in range(args.steps)]
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3 / args.steps
        nl, ms = plan.timing_read()
        plan.timing_enable(None)
        return res[-1], wall, nl // args.steps, ms / args.steps

    # momentum: Crank-Nicolson with QUICK convection, nu = 1e-3 (Re 300 on the sphere); the
    # 'momentum' class times the Jacobi sweeps only
    ut = [plan.empty() for _ in range(3)]
    mo, wall, nl, ms = timed("momentum", lambda: plan.momentum(
        u, pr["U_in"], pr["dt"], 1e-3, scheme="cn", cn_tol=1e-10, out=ut))
    rep = mo["report"]
    # per Jacobi sweep: read the iterate, u^n (advecting) and the right-hand side, write the
    # next iterate (3 components each, FP64): 12 words per cell, faces excluded
    its = rep.n_inner
    sweep_ms = ms / max(nl, 1)
    gbs = 96.0 * n_cells / (sweep_ms * 1e-3) / 1e9
    out["momentum"] = {"scheme": "crank-nicolson + QUICK, nu 1e-3", "ms_per_step": wall,
                       "iterations": its, "final_rel_res": rep.final_rel_res,
                       "kernel_launches": nl, "kernel_ms": ms,
                       "roofline": {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS,
                                    "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS,
                                    "alg_bytes_per_cell": 96,
                                    "note": "Jacobi sweep of the Crank-Nicolson system: read "
                                            "the iterate, u^n and the right-hand side, write "
                                            "the next iterate (FP64), faces excluded"}}
    log(f"[bench] momentum: {wall:.2f} ms/step, {its} sweeps, {gbs:.0f} GB/s per launch")
    # Lagrangian-particle forcing: the sphere's surface at one particle per h^2
    h = float(m.h().min())
    X, dV = sphere_particles((0.5, 0.5, 0.5), 0.15, h)
    Xd, dVd = dev(X), dev(dV)
    us = [plan.empty() for _ in range(3)]
    _, wall, nl, ms = timed("ib", lambda: plan.ib_force(u, Xd, pr["dt"], pr["rho"], dV=dVd,
                                                        out=us))
    out["ib_particles"] = {"particles": int(len(X)), "ms_per_call": wall, "kernel_ms": ms,
                           "particles_per_s": len(X) / (ms * 1e-3) if ms > 0 else None,
                           "note": "27 cells x 3 components gathered and spread per particle "
                                   "(FP64 atomics); the call also copies u~ to u* and reads "
                                   "the skip count back"}
    log(f"[bench] particles: {len(X)} in {ms * 1e3:.1f} us (kernel)")
    # checkpoint codec on the pressure of the projection step, 1e-4 of max |p|
    pp = plan.project(u, dev(pr["alpha"]), pr["U_in"], pr["dt"], pr["rho"])["p"]
    pmax = float(pp.abs().max())
    step = 2 * 1e-4 * pmax / 24.375
    buf = torch.empty(plan.compress_bound(), dtype=torch.uint8, device="cuda")
    s, wall_c, nl_c, ms_c = timed("codec", lambda: plan.compress(pp, step, out=buf))
    dec = plan.empty(torch.float64)
    _, wall_d, nl_d, ms_d = timed("codec", lambda: plan.decompress(s, out=dec))
    err = float((dec - pp).abs().max()) / pmax
    out["codec"] = {"field": "pressure, FP64", "step": step, "ratio": 8.0 * n_cells / s.numel(),
                    "max_rel_error": err, "compress_ms": wall_c, "compress_kernel_ms": ms_c,
                    "decompress_ms": wall_d, "decompress_kernel_ms": ms_d,
                    "compress_GBps": 8.0 * n_cells / (ms_c * 1e-3) / 1e9,
                    "decompress_GBps": 8.0 * n_cells / (ms_d * 1e-3) / 1e9}
    log(f"[bench] codec: ratio 1:{out['codec']['ratio']:.1f}, error {err:.1e}, compress "
        f"{ms_c:.3f} ms, decompress {ms_d:.3f} ms (kernels)")
    del buf, plan
    torch.cuda.empty_cache()
    return out


def run(args):
    import numpy as np
    import torch
    from paper_1808_04099_amd import Mesh, Plan

    pr, desc = workload(args.workload)
    m = pr["mesh"]
    n_cells = m.n_cells
    log(f"[bench] workload {desc}")
    mesh = Mesh(m)

    extra = {}
    for kv in args.opt:
        k, v = kv.split("=")
        extra[k] = float(v) if k in ("tol", "inner_tol") else int(v)

    def make(precision):
        plan = Plan(mesh, precision=precision, **{"tol": 1e-10, **extra})
        dt = torch.float32 if precision == "mixed_f32fields" else torch.float64
        u = [torch.from_numpy(np.ascontiguousarray(pr["u"][d]).reshape(-1)).to("cuda", dt)
             for d in range(3)]
        a = torch.from_numpy(np.ascontiguousarray(pr["alpha"]).reshape(-1)).to("cuda", dt)
        out = dict(u_new=[plan.empty() for _ in range(3)], p=plan.empty(torch.float64))
        return plan, u, a, out

    def step(plan, u, a, out):
        return plan.project(u, a, pr["U_in"], pr["dt"], pr["rho"], out=out)["report"]

    def timed_steps(plan, u, a, out, steps, timer_cls=None, every=1):
        if timer_cls:
            plan.timing_enable(timer_cls, every)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = [step(plan, u, a, out) for _ in range(steps)]
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        timing = plan.timing_read() if timer_cls else None
        if timer_cls:
            plan.timing_enable(None)
        return ms, reps, timing

    prec = args.precision
    plan, u, a, out = make(prec)
    s = 4 if prec != "fp64" else 8
    f = 4 if prec == "mixed_f32fields" else 8
    body = float((a.view(m.n_cubes, -1) != 0).any(dim=1).double().mean().item())
    for _ in range(args.warmup):
        rep = step(plan, u, a, out)
    torch.cuda.synchronize()
    # time each kernel class over two untimed steps (one class timed per step); the dominant
    # one is the streaming class with the largest share of the step
    dominant, best = args.kernel, -1.0
    class_ms = {}
    for cls in () if args.kernel else CLASSES:
        _, _, (nl, tot) = timed_steps(plan, u, a, out, 2, cls)
        nl, tot = nl // 2, tot / 2.0       # per step
        class_ms[cls] = {"launches": nl, "ms_per_step": tot}
        bpc = alg_bytes_per_cell(cls, s, f, body)
        if bpc is not None and nl > 0:
            gbs = bpc * level_cells(cls, n_cells, m.n) / (tot / nl * 1e-3) / 1e9
            class_ms[cls].update(alg_gbs=gbs, frac=gbs / PEAK_HBM_GBS)
        log(f"[bench] {cls}: {nl} launches, {tot:.3f} ms per step")
        if args.kernel is None and bpc is not None and tot > best:
            dominant, best = cls, tot
    # in the timed steps one launch of the dominant class in four is bracketed by events
    # (each event holds the stream for a few microseconds)
    ms, reps, (nl, tot) = timed_steps(plan, u, a, out, args.steps, dominant, every=4)
    rep = reps[-1]
    sweeps = plan.opts.pre_sweeps + plan.opts.post_sweeps
    per_iter = sweeps + 2              # smoothing sweeps + restriction residual + operator apply
    updates = n_cells * (rep.n_inner * per_iter + (rep.n_outer + 1) + 2)
    value = updates / (ms * 1e-3)
    avg_ms = tot / max(nl, 1)
    bpc = alg_bytes_per_cell(dominant, s, f, body)
    cells_dom = level_cells(dominant, n_cells, m.n)
    achieved = bpc * cells_dom / (avg_ms * 1e-3) / 1e9
    log(f"[bench] {prec}: {ms:.2f} ms/step, {rep.n_inner} inner its, {rep.n_outer} outer, "
        f"rel.res {rep.final_rel_res:.2e}; {dominant}: {avg_ms:.3f} ms/launch, "
        f"{achieved:.0f} GB/s")
    log("[bench] residual history: " + " ".join(f"{v:.1e}" for v in rep.history))
    result = {
        "metric": "Poisson cell-updates/s (mixed-precision projection to 1e-10)",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec != "fp64" else "f64",
        "data": "synthetic",
        "config": {"workload": desc, "cells": n_cells, "cubes": m.n_cubes,
                   "precision": prec, "tol": 1e-10, "parallelism": "single GPU"},
        "iterations": {"inner": rep.n_inner, "outer": rep.n_outer,
                       "final_rel_res": rep.final_rel_res,
                       "cell_updates_per_step": updates},
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": achieved,
                     "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS,
                     "traffic": measured_traffic(dominant, args.workload, prec),
                     "alg_bytes_per_launch": bpc * cells_dom, "alg_bytes_per_cell": bpc,
                     "launches": nl, "avg_launch_ms": avg_ms},
        "kernel_classes": class_ms,
    }
    if args.compare_fp64 and prec != "fp64":
        # keep this precision's result of the last timed step to compare with the FP64 one
        p_mixed = out["p"].clone()
        u_mixed = [x.to(torch.float64) for x in out["u_new"]]
        del plan, out
        torch.cuda.empty_cache()
        p64, u64, a64, o64 = make("fp64")
        for _ in range(max(1, args.warmup)):
            step(p64, u64, a64, o64)
        ms64, reps64, _ = timed_steps(p64, u64, a64, o64, args.steps)
        result["fp64_ms_per_step"] = ms64
        result["fp64_iterations"] = reps64[-1].n_inner
        result["fp64_final_rel_res"] = reps64[-1].final_rel_res
        result["mixed_speedup_vs_fp64"] = ms64 / ms
        # max-norm difference of this precision's result from the all-FP64 one, relative to
        # the largest value (both solves reach the same 1e-10 residual)
        rel = lambda a, b: float((a - b).abs().max() / b.abs().max())
        result["rel_diff_vs_fp64"] = {
            "p": rel(p_mixed, o64["p"]),
            "u_new": max(rel(u_mixed[d], o64["u_new"][d]) for d in range(3))}
        log(f"[bench] difference from the FP64 result: p {result['rel_diff_vs_fp64']['p']:.1e}, "
            f"u {result['rel_diff_vs_fp64']['u_new']:.1e}")
        log(f"[bench] fp64: {ms64:.2f} ms/step, {reps64[-1].n_inner} its; "
            f"mixed speed-up {ms64 / ms:.2f}x")
        del p64, o64
    if args.next_rows and args.workload in ("mixed_channel", "sphere_channel", "small_box"):
        result["next_rows"] = next_rows(pr, mesh, args)
    if args.copy_probe:
        cp = copy_probe()
        result["copy_probe"] = cp
        log(f"[bench] torch device copy: {cp['gbs']:.0f} GB/s (read + write of "
            f"{cp['bytes_per_copy'] // 2} bytes)")
    if args.cpu_baseline:
        log("[bench] timing the CPU oracle ...")
        cb = cpu_baseline(pr, args.cpu_seconds)
        result["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        result["cpu_baseline"]["oracle_projection_s"] = cb["oracle_projection_s"]
    print(json.dumps(result), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mixed_channel",
                    choices=["mixed_channel", "sphere_channel", "small_box", "multilevel"])
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed", "mixed_f32fields"])
    ap.add_argument("--kernel", default=None,
                    choices=[c for c in CLASSES if alg_bytes_per_cell(c, 4, 8) is not None],
                    help="timer class for the roofline (skips the per-class survey)")
    ap.add_argument("--no-compare-fp64", dest="compare_fp64", action="store_false")
    ap.add_argument("--no-cpu-baseline", dest="cpu_baseline", action="store_false")
    ap.add_argument("--no-copy-probe", dest="copy_probe", action="store_false",
                    help="skip the device-copy bandwidth probe")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-next-rows", dest="next_rows", action="store_false",
                    help="skip the momentum / particle / codec measurements")
    ap.add_argument("--opt", action="append", default=[],
                    help="solver option override key=value (e.g. coarse_iters=40)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only: the projection path is "
                                   "not sharded (see the multi-GPU design notes); use --gpus 1"}))
        sys.exit(2)
    run(args)


if __name__ == "__main__":
    main()
