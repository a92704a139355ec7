#!/usr/bin/env python3
"""Throughput of the two-phase Navier-Stokes time step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload c5] [--no-cpu-baseline]

A step is one whole pass of the hot path: the time step of the CFL rule on
the current velocity (ns_cfl_dt), level-set advection and
reinitialisation, properties, the momentum predictor, and the projection
solved by MG-preconditioned CG to ||b - A p|| <= 1e-10 ||b||.  The default
workload is the largest single-GPU tank, 512x256x256 cells (4 x 2 x 2 m,
33.5 M cells, 1 m water, JONSWAP waves Hs 0.2 m Tp 2 s, two cylinders
heaving at a prescribed velocity), in plain FP64, with synthetic seeded
inputs already resident in device memory when the timed region starts.

Printed: ONE JSON line with
  value        Mcell-steps/s over the K timed steps (cells x K / seconds)
  roofline     the dominant kernel (the finest-level red-black smoothing,
               one colour pass per launch): its algorithmic bytes per launch
               (48 B per cell per red-black sweep: beta on the three face
               arrays once, b, e read and e written once; 24 B per cell per
               colour pass) over its average duration from HIP events on
               the library's stream, against the published 8 TB/s; traffic
               from rocprofv3 counters, below the algorithmic bytes because
               face lines of one value are read from the line tables (the
               fraction of such lines is reported)
  step_roofline  the whole step's algorithmic bytes (380 B per cell outside
               the solve, 387 B per cell per FP64 CG iteration) over the
               measured step time
  phases       device time of each phase of a step (level set, predictor,
               projection set-up, CG, correction)
  configs      the FP64 step on the other tanks: 256x64 (2-D), 128x64x64,
               256x128x128
  projection_study  projection wall time and CG iterations to the same
               1e-10 true residual: FP64 V-cycle (zero and previous-pressure
               guesses), FP32 V-cycle (previous-pressure and learned guesses,
               inference included, and the per-step choice that runs the
               network only where it is measured to pay), the learned guess's
               break-even in CG iterations, the per-field difference of the
               FP32-V-cycle step from the FP64 one, the network forward's
               BF16 rate; on 512x256x256 and the two 256x128x128 tanks
  fsi_study, nwt_study, option_study  free heave, the numerical wave tank
               and the predictor's options on the 128x64x64 tank
  measured_ceilings  a 1 GiB device copy and an 8192^3 BF16 matrix product
  cpu_baseline the FP64 CPU oracle on the host's cores (OpenMP, static
               schedule) and on one thread, each on the first step of the
               same workload
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
MFMA_BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix peak, published

# HBM bytes per launch of the dominant kernel from two rocprofv3 --pmc
# passes: FETCH_SIZE x its copy-calibrated factor (1.9998) + WRITE_SIZE,
# medians over the run's dispatches (the finest-level colour pass at
# 512x256x256 with the line tables, 606; the fused sweep there, reading
# every face, 336).  Valid for those kernels as they are now and for that
# workload only; None elsewhere.
TRAFFIC_BYTES_PER_LAUNCH = {
    ("k_gs<double, true>", "c5"): 545528840,
    ("k_gs_rb_fine<double, 13>", "c5"): 2027212498,
}

# Algorithmic bytes per cell (FP64, 3-D; each array read or written once per
# pass): the passes outside the solve, and one FP64 CG iteration (vector work
# 120 + the V(2,2) cycle 267 over all levels).
STEP_BYTES_PER_CELL = 380.0
ITER_BYTES_PER_CELL_FP64 = 387.0
# one red-black sweep of the smoother reads the three face arrays of beta,
# b and e once and writes e once: 48 B per cell, 24 per colour pass
SWEEP_BYTES_PER_CELL_FP64 = 48.0
# the kernel the library's smoother timer measures (ns.TIME_SMOOTH0) and the
# part of one red-black sweep of the finest level that one launch does: the
# fused sweep where the library uses it (large 3-D grids), else one colour
# pass
# with --precision mixed, the FP32 instances of the same kernels (half the bytes)
SMOOTHER_KERNELS_FP32 = {True: ("k_gs_rb_fine<float, 13> (one red-black sweep, finest level)", 1.0),
                         False: ("k_gs<float, true> (one red-black colour pass, finest level)", 0.5)}
SMOOTHER_KERNELS = {True: ("k_gs_rb_fine<double, 13> (one red-black sweep, finest level)", 1.0),
                    False: ("k_gs<double, true> (one red-black colour pass, finest level)", 0.5)}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def line_table_fractions(S):
    """The fraction of the finest level's face lines (along x, per j, k)
    that the library reads from its line tables: every face of the line one
    value, bit for bit (an x-line: every interior face, both wall faces
    zero).  From the current coefficients, on the device."""
    import torch
    out = {}
    for k in ("bx", "by", "bz"):
        a = S.buffer(k).view(torch.int64)
        if k == "bx":
            inner = a[..., 1:-1]
            one = (inner == inner[..., :1]).all(-1) & (a[..., 0] == 0) & (a[..., -1] == 0)
        else:
            one = (a == a[..., :1]).all(-1)
        out[k] = round(float(one.double().mean()), 4)
    return out


def timed_steps(S, wl, steps: int, t0: float = 0.0):
    """`steps` whole steps, each with the time step of the CFL rule taken on
    the device from the current velocity; returns (t, iters, dts)."""
    t, iters, dts = t0, [], []
    for _ in range(steps):
        dt = S.cfl_dt(wl.cfl, wl.dt_max)
        st = S.step(dt, t)
        iters.append(st["iters"])
        dts.append(dt)
        t += dt
    return t, iters, dts


def run_gpu(args):
    import torch

    from paper_2206_07732_amd import inputs as I
    from paper_2206_07732_amd import ns

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU (the hot path runs only on the gfx950 library)")
    if not os.path.exists(ns.LIB_PATH):
        from paper_2206_07732_amd import build
        build.build()
    wl = I.workload(args.workload)
    f0 = I.make_fields(wl)
    ncell = wl.ncells

    # ---- main timed region: K whole FP64 steps
    dev = ns.device_fields(f0)
    mixed = args.precision == "mixed"
    S = ns.Solver(ns.params(wl, prec=ns.PREC_MIXED if mixed else ns.PREC_FP64), dev)
    t, _, _ = timed_steps(S, wl, args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t, iters, dts = timed_steps(S, wl, args.steps, t)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = ncell * args.steps / elapsed / 1e6
    log(f"[bench] {args.workload}: {ms_per_step:.3f} ms/step, {value:.1f} Mcell-steps/s, CG iters {iters}")

    # ---- where a step's time goes (device time per phase, three steps)
    S.phase_timing(True)
    ph = []
    for _ in range(3):
        dt = S.cfl_dt(wl.cfl, wl.dt_max)
        ph.append(S.step(dt, t)["t_ms"])
        t += dt
    S.phase_timing(False)
    names = ["level_set", "predictor", "projection_setup", "cg_solve", "correction", "step"]
    phases = {n: round(statistics.mean(p[q] for p in ph), 4) for q, n in enumerate(names)}
    log(f"[bench] phases (ms): {phases}")

    # ---- the dominant kernel: the finest-level red-black smoothing.  Its
    # average duration from HIP events around a batch of back-to-back
    # dispatches on the library's stream (the figure rocprofv3's kernel trace
    # reproduces, also for the dispatches inside steps), and from events
    # recorded with each dispatch inside steps (lower: there a sweep follows
    # the kernel that wrote its inputs, part of them still on chip).
    reps = 100
    tables = line_table_fractions(S) if S.face_tables() else None
    fused = S.fine_sweep()
    smoother_kernel, sweeps_per_launch = (SMOOTHER_KERNELS_FP32 if mixed else SMOOTHER_KERNELS)[fused]
    sweep_bytes = SWEEP_BYTES_PER_CELL_FP64 / (2 if mixed else 1)
    avg_ms = S.time_kernel(ns.TIME_SMOOTH0, reps)
    S.timing_enable(ns.TIME_SMOOTH0, 4096)
    for _ in range(2):
        dt = S.cfl_dt(wl.cfl, wl.dt_max)
        S.step(dt, t)
        t += dt
    kms, kn = S.timing_read()
    S.timing_enable(ns.TIME_SMOOTH0, 0)
    S.close()
    kbytes = sweep_bytes * sweeps_per_launch * ncell
    in_step_ms = kms / max(kn, 1)
    achieved = kbytes / (avg_ms * 1e-3) / 1e9
    achieved_in_step = kbytes / (in_step_ms * 1e-3) / 1e9
    traffic = TRAFFIC_BYTES_PER_LAUNCH.get((smoother_kernel.split(" (")[0], args.workload))
    roofline = {"kernel": smoother_kernel, "bound": "hbm", "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "traffic_over_algorithmic": round(traffic / kbytes, 3) if traffic else None,
                "bytes_per_launch": int(kbytes), "sweeps_per_launch": sweeps_per_launch,
                "bytes_per_cell_per_sweep": sweep_bytes,
                "avg_us": round(avg_ms * 1e3, 3), "launches": reps, "timing": "HIP events around "
                "a batch of back-to-back dispatches on the library's stream",
                "in_step_avg_us": round(in_step_ms * 1e3, 3), "in_step_launches": kn,
                "in_step_frac": round(achieved_in_step / HBM_PEAK_GBS, 4),
                "line_tables": tables}
    log(f"[bench] smoother: {avg_ms * 1e3:.2f} us per launch back to back ({achieved:.0f} GB/s, "
        f"{100 * achieved / HBM_PEAK_GBS:.1f}% of 8 TB/s); {in_step_ms * 1e3:.2f} us inside steps")
    mean_it = statistics.mean(iters)
    step_bytes = (STEP_BYTES_PER_CELL + mean_it * ITER_BYTES_PER_CELL_FP64) * ncell
    step_gbs = step_bytes / (ms_per_step * 1e-3) / 1e9
    step_roofline = {"bound": "hbm", "achieved": round(step_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(step_gbs / HBM_PEAK_GBS, 4), "bytes_per_step": int(step_bytes),
                     "bytes_per_cell": STEP_BYTES_PER_CELL + mean_it * ITER_BYTES_PER_CELL_FP64,
                     "mean_cg_iters": mean_it}
    if mixed:   # the byte counts above are the FP64 cycle's
        step_roofline = {"note": "counted for the FP64 step only"}
    else:
        log(f"[bench] whole step: {step_gbs:.0f} GB/s algorithmic ({100 * step_gbs / HBM_PEAK_GBS:.1f}% of 8 TB/s)")
    ceil = measured_ceilings()
    roofline["copy_ceiling_gbs"] = ceil["copy_gbs"]
    roofline["frac_of_copy"] = round(achieved / ceil["copy_gbs"], 4)
    log(f"[bench] measured ceilings: device copy {ceil['copy_gbs']:.0f} GB/s, BF16 GEMM "
        f"{ceil['bf16_gemm_tflops']:.0f} TFLOP/s")
    config = {"workload": wl.name, "grid": [wl.nx, wl.ny, wl.nz], "cells": ncell, "h": wl.h,
              "dt": "CFL rule on the current velocity each step", "cfl": wl.cfl,
              "dt_range": [min(dts), max(dts)],
              "solver": "flexible PCG, V(2,2) red-black GS, " + ("FP32 V-cycle in FP64 CG" if mixed else "FP64"),
              "rtol": 1e-10,
              "mg_levels": ns.num_levels(wl.nx, wl.ny, wl.nz)}
    return {"value": value, "ms_per_step": ms_per_step, "iters": iters, "roofline": roofline,
            "step_roofline": step_roofline, "phases": phases, "config": config, "wl": wl, "f0": f0,
            "ceilings": ceil}


def measured_ceilings():
    """What the device reaches on plain work, as context for the published
    peaks: a 1 GiB device-to-device copy (bytes read + written per second)
    and an 8192^3 BF16 matrix product (torch, i.e. the vendor library)."""
    import torch
    n = (1 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * 8 * n * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    m = 8192
    g = torch.Generator(device="cuda").manual_seed(0)
    x = torch.randn(m, m, device="cuda", dtype=torch.bfloat16, generator=g)
    y = torch.randn(m, m, device="cuda", dtype=torch.bfloat16, generator=g)
    for _ in range(2):
        z = torch.matmul(x, y)
    e0.record()
    for _ in range(5):
        z = torch.matmul(x, y)
    e1.record()
    torch.cuda.synchronize()
    gemm = 2.0 * m ** 3 * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e12
    del x, y, z
    torch.cuda.empty_cache()
    return {"copy_gbs": round(copy_gbs, 1), "bf16_gemm_tflops": round(gemm, 1)}


def config_line(name: str, steps: int, warmup: int):
    """The FP64 step on another tank, timed like the main one."""
    import torch

    from paper_2206_07732_amd import inputs as I
    from paper_2206_07732_amd import ns
    wl = I.workload(name)
    S = ns.Solver(ns.params(wl), ns.device_fields(I.make_fields(wl)))
    t, _, _ = timed_steps(S, wl, warmup)
    torch.cuda.synchronize()
    a = time.perf_counter()
    t, iters, _ = timed_steps(S, wl, steps, t)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - a) / steps
    S.close()
    out = {"workload": wl.name, "cells": wl.ncells, "steps": steps, "ms_per_step": round(ms, 4),
           "mcell_steps_per_s": round(wl.ncells / (ms * 1e-3) / 1e6, 3), "cg_iters": iters}
    log(f"[bench] {name}: {ms:.3f} ms/step, {out['mcell_steps_per_s']} Mcell-steps/s, iters {iters}")
    return out


# FLOPs of one inference of the learned-guess network per voxel of the full
# grid: 2 * 27 * C_in * C_out per output voxel and layer (first layer with its
# 4 real input channels; levels 2 and 3 hold 1/8 and 1/64 of the voxels), plus
# the 1x1x1 head.
NET_FLOP_PER_VOXEL = (2 * 27 * 4 * 16 + 2 * 27 * 48 * 16 + 2 * 16) + (2 * 27 * 16 * 32 + 2 * 27 * 96 * 32) / 8 + \
    (2 * 27 * 32 * 64) / 64


def projection_study(name: str, steps: int, warmup: int, weights: str):
    """Projection wall time and CG iterations to the same 1e-10 true residual
    on one workload for: FP64 V-cycle from zero and from the previous
    pressure, FP32 V-cycle from the previous pressure, FP32 V-cycle from the
    learned guess (network inference included in the time), and FP32 V-cycle
    with the guess chosen per step (NS_X0_AUTO: inference only where it is
    measured to pay).  The learned guess's break-even: the CG iterations its
    inference costs at the FP32 V-cycle's time per iteration, against the
    iterations it saves.  Also the per-field difference of the FP32-V-cycle
    step from the FP64 one, both taken from the same state, and the network
    forward's matrix-core rate."""
    import numpy as np
    import torch

    from paper_2206_07732_amd import inputs as I
    from paper_2206_07732_amd import ns

    wl = I.workload(name)
    f0 = I.make_fields(wl)
    net = None
    if weights and os.path.exists(weights):
        net = ns.Net(wl.nx, wl.ny, wl.nz)
        net.set_params(np.load(weights, allow_pickle=False))
    out = {"workload": wl.name, "grid": [wl.nx, wl.ny, wl.nz], "steps_timed": steps, "rtol": 1e-10,
           "weights": os.path.relpath(weights, ROOT) if net is not None else None}
    variants = [("fp64", "zero"), ("fp64", "prev"), ("mixed", "prev")]
    if net is not None:
        variants += [("mixed", "learned"), ("mixed", "auto")]
    for prec, x0 in variants:
        dev = ns.device_fields(f0)
        S = ns.Solver(ns.params(wl, prec=ns.PREC_FP64 if prec == "fp64" else ns.PREC_MIXED,
                                x0={"zero": ns.X0_ZERO, "prev": ns.X0_PREV, "learned": ns.X0_LEARNED,
                                    "auto": ns.X0_AUTO}[x0]), dev)
        if x0 in ("learned", "auto"):
            S.attach_net(net)
        t, _, _ = timed_steps(S, wl, warmup)
        ms, its, r0, res, used = [], [], [], [], []
        for _ in range(steps):
            dt = S.cfl_dt(wl.cfl, wl.dt_max)
            S.levelset_advect_reinit(dt)
            S.momentum_step(dt, t + dt)
            torch.cuda.synchronize()
            a = time.perf_counter()
            st = S.projection_solve(dt)
            ms.append(1e3 * (time.perf_counter() - a))
            its.append(st["iters"])
            r0.append(st["rel_resid0"])
            res.append(st["true_rel_resid"])
            used.append(st["x0_used"])
            t += dt
        out[f"{prec}+{x0}"] = {"ms_median": round(statistics.median(ms), 4), "iters": its,
                               "mean_rel_resid0": float(np.mean(r0)), "max_true_rel_resid": max(res)}
        if x0 == "auto":
            out[f"{prec}+{x0}"].update({"ms_mean": round(statistics.mean(ms), 4), "x0_used": used,
                                        "gain_iters": round(st["x0_gain"], 3)})
        log(f"[bench] {wl.name[:6]} projection {prec}+{x0}: {statistics.median(ms):.3f} ms, iters {its}")
        S.close()
    base = out["fp64+prev"]["ms_median"]
    for k in ("mixed+prev", "mixed+learned", "mixed+auto"):
        if k in out:
            out[k]["speedup_vs_fp64_prev"] = round(base / out[k]["ms_median"], 3)
    if "mixed+learned" in out:
        # what inference costs in CG iterations of the FP32 V-cycle, and what it saves
        mp, ml = out["mixed+prev"], out["mixed+learned"]
        t_it = mp["ms_median"] / statistics.mean(mp["iters"])
        saved = statistics.mean(mp["iters"]) - statistics.mean(ml["iters"])
        cost_ms = ml["ms_median"] - mp["ms_median"] + saved * t_it
        out["learned_break_even"] = {"ms_per_cg_iter": round(t_it, 4), "inference_ms": round(cost_ms, 4),
                                     "break_even_iters": round(cost_ms / t_it, 2), "saved_iters": round(saved, 2)}
        log(f"[bench] {wl.name[:6]} learned guess: inference {cost_ms:.3f} ms = {cost_ms / t_it:.2f} CG "
            f"iterations, saves {saved:.2f}")
    # per-field difference of one step with the FP32 V-cycle from the FP64 one
    fields = {}
    for prec in (ns.PREC_FP64, ns.PREC_MIXED):
        dev = ns.device_fields(f0)
        S = ns.Solver(ns.params(wl, prec=prec), dev)
        dt = S.cfl_dt(wl.cfl, wl.dt_max)
        S.step(dt, 0.0)
        torch.cuda.synchronize()
        fields[prec] = {k: v.clone() for k, v in dev.items()}
        S.close()
    err = {}
    for k in ("p", "u", "v", "w", "sigma"):
        a, b = fields[ns.PREC_MIXED][k], fields[ns.PREC_FP64][k]
        nrm = float(torch.linalg.vector_norm(b))
        err[k] = {"rel_l2": float(torch.linalg.vector_norm(a - b)) / nrm if nrm > 0 else 0.0,
                  "max_abs": float((a - b).abs().max())}
    del fields
    out["mixed_vs_fp64_one_step"] = err
    if net is not None:
        feat = torch.randn((4, wl.nz, wl.ny, wl.nx), dtype=torch.float32, device="cuda")
        for _ in range(2):
            net.forward(feat)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 10
        with torch.cuda.stream(net.stream):
            e0.record()
            for _ in range(reps):
                net.forward(feat)
            e1.record()
        torch.cuda.synchronize()
        fwd_ms = e0.elapsed_time(e1) / reps
        tflops = NET_FLOP_PER_VOXEL * wl.ncells / (fwd_ms * 1e-3) / 1e12
        out["net_forward"] = {"ms": round(fwd_ms, 4), "flop_per_voxel": NET_FLOP_PER_VOXEL,
                              "achieved_tflops": round(tflops, 1), "peak_tflops": MFMA_BF16_PEAK_TFLOPS,
                              "frac": round(tflops / MFMA_BF16_PEAK_TFLOPS, 4)}
        log(f"[bench] network forward {fwd_ms:.3f} ms ({tflops:.0f} TFLOP/s BF16)")
        net.close()
    torch.cuda.empty_cache()
    return out


def option_overrides(opt: str) -> dict:
    """'consistent', 'cnN' or both joined by '+' -> workload overrides."""
    over = {}
    for o in opt.split("+"):
        if o == "consistent":
            over["consistent"] = 1
        elif o.startswith("cn") and o[2:].isdigit():
            over["cn_sweeps"] = int(o[2:])
        else:
            raise SystemExit(f"unknown predictor option {o!r} (consistent, cnN)")
    return over


def variant_study(name: str, steps: int, warmup: int, base: dict, label: str = "", **over):
    """A variant of a tank (free heave, a numerical wave tank, or an option
    of the predictor): K whole steps after W warm-up steps, timed like the
    main run; base is the same grid's plain run for comparison.  For a free
    body also its heave range and its force over its weight."""
    import torch
    from paper_2206_07732_amd import inputs as I, ns
    wl = I.workload(name, **over)
    S = ns.Solver(ns.params(wl), ns.device_fields(I.make_fields(wl)))
    t, _, _ = timed_steps(S, wl, warmup)
    torch.cuda.synchronize()
    free = any(b.free_heave for b in wl.bodies)
    zeta, fz, iters, cn = [], [], [], []
    a = time.perf_counter()
    for _ in range(steps):
        dt = S.cfl_dt(wl.cfl, wl.dt_max)
        st = S.step(dt, t)
        t += dt
        iters.append(st["iters"])
        cn.append(st["cn_sweeps"])
        if free:
            b = S.body_state(0)       # host state: no device work
            zeta.append(b["zeta"])
            fz.append(b["F"][2])
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - a) / steps
    S.close()
    out = {
        "workload": wl.name + (f" [{label}]" if label else ""),
        "steps": steps,
        "ms_per_step": round(ms, 4),
        "mcell_steps_per_s": round(wl.ncells / (ms * 1e-3) / 1e6, 3),
        "cg_iters": iters,
        "ms_per_cg_iter": round(ms / statistics.mean(iters), 4),
        "base_ms_per_step": base["ms_per_step"],
        "base_ms_per_cg_iter": round(base["ms_per_step"] / statistics.mean(base["cg_iters"]), 4),
    }
    if wl.cn_sweeps:
        out["cn_sweeps"] = cn
    if free:
        mg = wl.bodies[0].mass * wl.g
        out["zeta_range_m"] = [round(min(zeta), 6), round(max(zeta), 6)]
        out["fz_over_mg_range"] = [round(min(fz) / mg, 4), round(max(fz) / mg, 4)]
    log(f"[bench] {name}{' ' + label if label else ''}: {ms:.3f} ms/step ({out['ms_per_cg_iter']} ms per CG "
        f"iteration; plain tank {out['base_ms_per_cg_iter']}), iters {iters}"
        + (f", zeta in {out['zeta_range_m']} m, Fz/mg in {out['fz_over_mg_range']}" if free else ""))
    return out


def run_cpu_baseline(wl, f0, steps: int):
    """The oracle as it stands on the first `steps` steps of the workload from
    its initial condition (each with the oracle's own CFL rule): on all host
    cores (OpenMP build, static schedule), then on one thread."""
    from oracle import oracle as O
    out = {}
    for label, omp in (("all_cores", True), ("one_thread", False)):
        O.use_openmp(omp)
        O.lib()
        P = O.params(wl)
        f, t = f0, 0.0
        iters = []
        t0 = time.perf_counter()
        for _ in range(steps):
            dt = O.cfl_dt(P, f, wl.cfl, wl.dt_max)
            f, st, rc = O.step(P, f, dt, t)
            iters.append(st["iters"])
            t += dt
        el = time.perf_counter() - t0
        out[label] = {"value": round(wl.ncells * steps / el / 1e6, 4), "seconds": round(el, 2),
                      "cg_iters": iters}
        log(f"[bench] cpu oracle ({label}): {out[label]['value']} Mcell-steps/s, {el:.1f} s for {steps} step(s)")
    O.use_openmp(False)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    return {"value": out["all_cores"]["value"], "unit": "Mcell-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"the first {steps} step(s) of the same workload ({wl.nx}x{wl.ny}x{wl.nz}) from its "
                      f"initial condition, FP64, OpenMP static schedule on {threads} threads; "
                      f"{out['all_cores']['seconds']} s",
            "one_thread": {**out["one_thread"], "cores": 1}, "all_cores": out["all_cores"], "host": host_cpu()}


def host_cpu() -> str:
    """CPU model and logical core count of the host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model}, {os.cpu_count()} logical cores"


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c5")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64",
                    help="the main timed step's V-cycle: FP64 (the default), or FP32 inside the FP64 CG")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=1)
    ap.add_argument("--configs", default="c1,c2,c3",
                    help="comma-separated tanks whose FP64 step is also timed; 'none' skips them")
    ap.add_argument("--projection-workload", default="c5,c3,c4eval",
                    help="comma-separated workloads of the projection study (FP64 vs FP32 V-cycle vs learned "
                         "guess); 'none' skips it")
    ap.add_argument("--projection-steps", type=int, default=10)
    ap.add_argument("--side-workload", default="c2", help="tank of the free-heave, wave-tank and option studies")
    ap.add_argument("--fsi-workload", default="c2fsi",
                    help="workload of the free-heave study (a free body on the side tank); 'none' skips it")
    ap.add_argument("--nwt-workload", default="c2nwt",
                    help="workload of the wave-tank study (the side grid with generation and damping zones); "
                         "'none' skips it")
    ap.add_argument("--option-studies", default="consistent,cn3",
                    help="comma-separated predictor options timed on the side tank: 'consistent' "
                         "(consistent mass/momentum transport), 'cnN' (Crank-Nicolson viscous term, N Jacobi "
                         "sweeps per convergence check), or both joined by '+'; 'none' skips them")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_2206_07732_amd", "weights", "guess_c4.npy"))
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run a plain device copy of this size (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(how the step would shard is described in the design notes). Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    r = run_gpu(args)
    if args.copy_calibration_mib > 0:
        import torch
        n = args.copy_calibration_mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log(f"[bench] copy calibration: 3 x {args.copy_calibration_mib} MiB device copies")
    configs = None
    if args.configs != "none":
        steps = {"c1": 10, "c2": 20, "c3": 10}
        configs = [config_line(c, steps.get(c, 10), 3) for c in args.configs.split(",")]
    study = None
    if args.projection_workload != "none":
        study = [projection_study(w, args.projection_steps, 2, args.weights)
                 for w in args.projection_workload.split(",")]
    side = None
    if args.fsi_workload != "none" or args.nwt_workload != "none" or args.option_studies != "none":
        side = next((c for c in configs or [] if c["workload"].startswith(args.side_workload + ":")), None) \
            or config_line(args.side_workload, 20, 3)
    fsi = variant_study(args.fsi_workload, 20, 3, side) if args.fsi_workload != "none" else None
    nwt = variant_study(args.nwt_workload, 20, 3, side) if args.nwt_workload != "none" else None
    opts = None
    if args.option_studies != "none":
        opts = [variant_study(args.side_workload, 20, 3, side, label=o, **option_overrides(o))
                for o in args.option_studies.split(",")]
    cpu = None
    if not args.no_cpu_baseline:
        cpu = run_cpu_baseline(r["wl"], r["f0"], args.cpu_steps)
    out = {
        "metric": "Mcell-steps/s + projection time @1e-10 resid: FP64 MG-CG vs mixed-prec+learned",
        "value": round(r["value"], 3),
        "unit": "Mcell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": r["config"],
        "cg_iters": r["iters"],
        "roofline": r["roofline"],
        "step_roofline": r["step_roofline"],
        "phases_ms": r["phases"],
        "configs": configs,
        "projection_study": study,
        "fsi_study": fsi,
        "nwt_study": nwt,
        "option_study": opts,
        "measured_ceilings": r["ceilings"],
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
