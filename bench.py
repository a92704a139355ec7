#!/usr/bin/env python3
"""Throughput of the two-phase Navier-Stokes time step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload c2] [--no-cpu-baseline]

A step is one whole pass of the hot path: level-set advection and
reinitialisation, properties, the momentum predictor, and the projection
solved by MG-preconditioned CG to ||b - A p|| <= 1e-10 ||b||.  The default
workload is the 3-D tank of 128x64x64 cells (4 x 2 x 2 m, 1 m water,
second-order Stokes wave a = 0.05 m, T = 1.2 s, fixed cylinder buoy) in
plain FP64, with synthetic seeded inputs already resident in device memory
when the timed region starts.

Printed: ONE JSON line with
  value        Mcell-steps/s over the K timed steps (cells x K / seconds)
  projection   projection wall time and CG iterations on the same workload,
               FP64 V-cycle vs FP32 V-cycle inside FP64 CG, both to the same
               1e-10 residual
  projection_study  the same on the 256x128x128 tanks (JONSWAP waves, and a
               held-out draw of the learned guess's Airy-wave training runs)
               for the FP64 V-cycle (zero and previous-pressure guesses) and
               the FP32 V-cycle (previous-pressure and learned guesses,
               inference included), the per-field difference of the
               FP32-V-cycle step from the FP64 one, and the network forward's
               BF16 rate
  fsi_study    free heave (force of eqn_int_fh, heave of eqn_newton_u) on the
               same tank with the cylinder free: whole ns_step calls timed the
               same way, against the fixed-body step, with the heave range and
               the force over the body's weight
  nwt_study    the same grid as a numerical wave tank (Airy waves generated at
               the inlet, generation and damping zones, vorticity damping),
               timed the same way
  option_study the main workload with the predictor's options: consistent
               mass/momentum transport, and the Crank-Nicolson viscous term
               (N Jacobi sweeps), timed the same way
  roofline     the finest-level smoother pass (the dominant kernel): its
               algorithmic bytes per launch over its average duration, the
               duration taken from HIP events recorded with each dispatch;
               against the published 8 TB/s and a measured device copy
  measured_ceilings  a 1 GiB device copy and an 8192^3 BF16 matrix product
               timed on the device, beside the published peaks
  cpu_baseline the FP64 CPU oracle, single-threaded, on a bounded sample of
               the same workload
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

# HBM bytes per launch of the finest smoother pass from rocprofv3 counters
# (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 KiB, the factors from a 256 MiB device
# copy measured in the same runs); None until taken for the current kernel.
TRAFFIC_BYTES_PER_LAUNCH = 19988958   # profiles/c2_smoother_hbm_counters.md


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def smoother_bytes_per_cell(prec: int) -> float:
    """Algorithmic bytes per cell of one colour pass of red-black Gauss-Seidel:
    beta on the three face arrays (every face touches a cell of each colour),
    b and the new e of that colour's half of the cells, and the old e of the
    other colour's half (its neighbours).  FP64: 24 + 4 + 4 + 4 = 36 B."""
    w = 8 if prec == 0 else 4
    return 3 * w + 0.5 * w + 0.5 * w + 0.5 * w


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
    dt = I.cfl_dt(wl, f0)
    ncell = wl.ncells

    # ---- main timed region: K whole FP64 steps
    dev = ns.device_fields(f0)
    S = ns.Solver(ns.params(wl, prec=ns.PREC_FP64), dev)
    t = 0.0
    for _ in range(args.warmup):
        S.step(dt, t)
        t += dt
    torch.cuda.synchronize()
    iters = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = S.step(dt, t)
        iters.append(st["iters"])
        t += dt
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = ncell * args.steps / elapsed / 1e6
    log(f"[bench] {args.workload}: {ms_per_step:.3f} ms/step, {value:.1f} Mcell-steps/s, CG iters {iters}")

    # ---- dominant kernel: the finest-level smoother pass.  Its average
    # duration is taken from HIP events around a batch of back-to-back
    # dispatches (amortising the events' own cost); the per-dispatch event
    # figure from inside real steps is reported beside it.
    reps = 200
    avg_ms = S.time_kernel(ns.TIME_SMOOTH0, reps)
    S.timing_enable(ns.TIME_SMOOTH0, 4096)
    for _ in range(2):
        S.step(dt, t)
        t += dt
    kms, kn = S.timing_read()
    S.timing_enable(ns.TIME_SMOOTH0, 0)
    kbytes = smoother_bytes_per_cell(0) * ncell
    achieved = kbytes / (avg_ms * 1e-3) / 1e9
    roofline = {"kernel": "k_gs<double, true> (one red-black colour pass, finest level)",
                "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": TRAFFIC_BYTES_PER_LAUNCH,
                "avg_us": round(avg_ms * 1e3, 3), "timed_launches": reps,
                "bytes_per_launch": int(kbytes),
                "in_step_event_avg_us": round(kms / max(kn, 1) * 1e3, 3), "in_step_launches": kn}
    log(f"[bench] smoother pass: avg {avg_ms*1e3:.2f} us over {reps} back-to-back launches "
        f"({achieved:.0f} GB/s); in-step per-dispatch events {kms/max(kn,1)*1e3:.2f} us over {kn}")
    S.close()
    ceil = measured_ceilings()
    roofline["copy_ceiling_gbs"] = ceil["copy_gbs"]
    roofline["frac_of_copy"] = round(achieved / ceil["copy_gbs"], 4)
    log(f"[bench] measured ceilings: device copy {ceil['copy_gbs']:.0f} GB/s, BF16 GEMM "
        f"{ceil['bf16_gemm_tflops']:.0f} TFLOP/s; smoother pass at {100 * achieved / ceil['copy_gbs']:.0f}% of the copy")

    # ---- projection time to 1e-10, FP64 V-cycle vs FP32 V-cycle in FP64 CG
    proj = {}
    for name, prec in (("fp64", ns.PREC_FP64), ("mixed", ns.PREC_MIXED)):
        d = ns.device_fields(f0)
        Sp = ns.Solver(ns.params(wl, prec=prec), d)
        tt = 0.0
        for _ in range(args.warmup):
            Sp.step(dt, tt)
            tt += dt
        ms, its, res = [], [], []
        for _ in range(max(3, min(args.steps, 10))):
            Sp.levelset_advect_reinit(dt)
            Sp.momentum_step(dt, tt + dt)
            torch.cuda.synchronize()
            a = time.perf_counter()
            st = Sp.projection_solve(dt)
            ms.append(1e3 * (time.perf_counter() - a))
            its.append(st["iters"])
            res.append(st["true_rel_resid"])
            tt += dt
        proj[name] = {"ms_median": round(statistics.median(ms), 4), "iters": its,
                      "max_true_rel_resid": max(res)}
        Sp.close()
    proj["speedup_mixed_vs_fp64"] = round(proj["fp64"]["ms_median"] / proj["mixed"]["ms_median"], 3)
    log(f"[bench] projection fp64 {proj['fp64']['ms_median']:.3f} ms, mixed {proj['mixed']['ms_median']:.3f} ms")

    config = {"workload": wl.name, "grid": [wl.nx, wl.ny, wl.nz], "cells": ncell, "h": wl.h,
              "dt": dt, "cfl": wl.cfl, "solver": "flexible PCG, V(2,2) red-black GS, FP64",
              "rtol": 1e-10, "mg_levels": ns.num_levels(wl.nx, wl.ny, wl.nz)}
    return {"value": value, "ms_per_step": ms_per_step, "iters": iters, "roofline": roofline,
            "projection": proj, "config": config, "wl": wl, "f0": f0, "dt": dt, "ceilings": ceil}


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


# FLOPs of one inference of the learned-guess network per voxel of the full
# grid: 2 * 27 * C_in * C_out per output voxel and layer (first layer with its
# 4 real input channels; levels 2 and 3 hold 1/8 and 1/64 of the voxels), plus
# the 1x1x1 head.
NET_FLOP_PER_VOXEL = (2 * 27 * 4 * 16 + 2 * 27 * 48 * 16 + 2 * 16) + (2 * 27 * 16 * 32 + 2 * 27 * 96 * 32) / 8 + \
    (2 * 27 * 32 * 64) / 64
MFMA_BF16_PEAK_TFLOPS = 2500.0   # MI355X dense BF16 matrix peak, published


def projection_study(name: str, steps: int, warmup: int, weights: str):
    """Projection wall time and CG iterations to the same 1e-10 true residual
    on one workload for: FP64 V-cycle from zero and from the previous
    pressure, FP32 V-cycle from the previous pressure, and FP32 V-cycle from
    the learned guess (network inference included in the time).  Also the
    per-field difference of the FP32-V-cycle step from the FP64 one, both
    taken from the same state, and the network forward's matrix-core rate."""
    import numpy as np
    import torch

    from paper_2206_07732_amd import inputs as I
    from paper_2206_07732_amd import ns

    wl = I.workload(name)
    f0 = I.make_fields(wl)
    dt = I.cfl_dt(wl, f0)
    net = None
    if weights and os.path.exists(weights):
        net = ns.Net(wl.nx, wl.ny, wl.nz)
        net.set_params(np.load(weights, allow_pickle=False))
    out = {"workload": wl.name, "grid": [wl.nx, wl.ny, wl.nz], "steps_timed": steps, "rtol": 1e-10,
           "weights": os.path.relpath(weights, ROOT) if net is not None else None}
    variants = [("fp64", "zero"), ("fp64", "prev"), ("mixed", "prev")]
    if net is not None:
        variants.append(("mixed", "learned"))
    for prec, x0 in variants:
        dev = ns.device_fields(f0)
        S = ns.Solver(ns.params(wl, prec=ns.PREC_FP64 if prec == "fp64" else ns.PREC_MIXED,
                                x0={"zero": ns.X0_ZERO, "prev": ns.X0_PREV, "learned": ns.X0_LEARNED}[x0]), dev)
        if x0 == "learned":
            S.attach_net(net)
        t = 0.0
        for _ in range(warmup):
            S.step(dt, t)
            t += dt
        ms, its, r0, res = [], [], [], []
        for _ in range(steps):
            S.levelset_advect_reinit(dt)
            S.momentum_step(dt, t + dt)
            torch.cuda.synchronize()
            a = time.perf_counter()
            st = S.projection_solve(dt)
            ms.append(1e3 * (time.perf_counter() - a))
            its.append(st["iters"])
            r0.append(st["rel_resid0"])
            res.append(st["true_rel_resid"])
            t += dt
        out[f"{prec}+{x0}"] = {"ms_median": round(statistics.median(ms), 4), "iters": its,
                               "mean_rel_resid0": float(np.mean(r0)), "max_true_rel_resid": max(res)}
        log(f"[bench] {wl.name[:3]} projection {prec}+{x0}: {statistics.median(ms):.3f} ms, iters {its}")
        S.close()
    base = out["fp64+prev"]["ms_median"]
    for k in ("mixed+prev", "mixed+learned"):
        if k in out:
            out[k]["speedup_vs_fp64_prev"] = round(base / out[k]["ms_median"], 3)
    # per-field difference of one step with the FP32 V-cycle from the FP64 one
    fields = {}
    for prec in (ns.PREC_FP64, ns.PREC_MIXED):
        dev = ns.device_fields(f0)
        S = ns.Solver(ns.params(wl, prec=prec), dev)
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


def variant_study(name: str, steps: int, warmup: int, fixed: dict, label: str = "", **over):
    """A variant of the main tank (free heave, a numerical wave tank, or an
    option of the predictor): K whole ns_step calls after W warm-up steps;
    fixed is the main run on the same grid for comparison.  For a free body
    also its heave range and its force over its weight."""
    import torch
    from paper_2206_07732_amd import inputs as I, ns
    wl = I.workload(name, **over)
    f = I.make_fields(wl)
    dt = I.cfl_dt(wl, f)
    S = ns.Solver(ns.params(wl), ns.device_fields(f))
    t = 0.0
    for _ in range(warmup):
        S.step(dt, t)
        t += dt
    torch.cuda.synchronize()
    free = any(b.free_heave for b in wl.bodies)
    zeta, fz, iters = [], [], []
    a = time.perf_counter()
    for _ in range(steps):
        st = S.step(dt, t)
        t += dt
        iters.append(st["iters"])
        if free:
            b = S.body_state(0)       # host state: no device work
            zeta.append(b["zeta"])
            fz.append(b["F"][2])
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - a) / steps
    S.close()
    ncell = wl.nx * wl.ny * wl.nz
    out = {
        "workload": wl.name + (f" [{label}]" if label else ""),
        "steps": steps,
        "ms_per_step": round(ms, 4),
        "mcell_steps_per_s": round(ncell * steps / (ms * steps * 1e-3) / 1e6, 3),
        "cg_iters": iters,
        "ms_per_cg_iter": round(ms / statistics.mean(iters), 4),
        "main_ms_per_step": round(fixed["ms_per_step"], 4),
        "main_ms_per_cg_iter": round(fixed["ms_per_step"] / statistics.mean(fixed["iters"]), 4),
    }
    if free:
        mg = wl.bodies[0].mass * wl.g
        out["zeta_range_m"] = [round(min(zeta), 6), round(max(zeta), 6)]
        out["fz_over_mg_range"] = [round(min(fz) / mg, 4), round(max(fz) / mg, 4)]
    log(f"[bench] {name}{' ' + label if label else ''}: {ms:.3f} ms/step ({out['ms_per_cg_iter']} ms per CG iteration; main tank "
        f"{out['main_ms_per_cg_iter']})" + (f", zeta in {out['zeta_range_m']} m, Fz/mg in {out['fz_over_mg_range']}"
                                             if free else ""))
    return out


def run_cpu_baseline(wl, f0, dt, seconds: float):
    """The oracle as it stands, single-threaded, for about `seconds`."""
    from oracle import oracle as O
    O.lib()
    P = O.params(wl)
    f, t, n, iters = f0, 0.0, 0, []
    t0 = time.perf_counter()
    while True:
        f, st, rc = O.step(P, f, dt, t)
        iters.append(st["iters"])
        t += dt
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds or n >= wl.steps:
            break
    return {"value": round(wl.ncells * n / el / 1e6, 4), "unit": "Mcell-steps/s", "cores": 1,
            "kind": "oracle", "sample": f"first {n} step(s) of the same workload from its initial "
                                        f"condition, {el:.1f} s, one thread",
            "cg_iters": iters, "host": host_cpu()}


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
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--projection-workload", default="c3,c4eval",
                    help="comma-separated workloads of the projection study (FP64 vs FP32 V-cycle vs learned "
                         "guess); 'none' skips it")
    ap.add_argument("--projection-steps", type=int, default=20)
    ap.add_argument("--fsi-workload", default="c2fsi",
                    help="workload of the free-heave study (a free body on the main tank); 'none' skips it")
    ap.add_argument("--nwt-workload", default="c2nwt",
                    help="workload of the wave-tank study (the main grid with generation and damping zones); "
                         "'none' skips it")
    ap.add_argument("--option-studies", default="consistent,cn3",
                    help="comma-separated predictor options timed on the main workload: 'consistent' "
                         "(consistent mass/momentum transport), 'cnN' (Crank-Nicolson viscous term by N "
                         "Jacobi sweeps), or both joined by '+'; 'none' skips them")
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
        log(f"[bench] copy calibration: 3 x {args.copy_calibration_mib} MiB device copies")
    study = None
    if args.projection_workload != "none":
        study = [projection_study(w, args.projection_steps, 2, args.weights)
                 for w in args.projection_workload.split(",")]
    fsi = None
    if args.fsi_workload != "none":
        fsi = variant_study(args.fsi_workload, args.steps, args.warmup, r)
    nwt = None
    if args.nwt_workload != "none":
        nwt = variant_study(args.nwt_workload, args.steps, args.warmup, r)
    opts = None
    if args.option_studies != "none":
        opts = [variant_study(args.workload, args.steps, args.warmup, r, label=o, **option_overrides(o))
                for o in args.option_studies.split(",")]
    cpu = None
    if not args.no_cpu_baseline:
        cpu = run_cpu_baseline(r["wl"], r["f0"], r["dt"], args.cpu_seconds)
        log(f"[bench] cpu oracle {cpu['value']} Mcell-steps/s ({cpu['sample']})")
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
        "dtype": "f64",
        "data": "synthetic",
        "config": r["config"],
        "cg_iters": r["iters"],
        "projection": r["projection"],
        "projection_study": study,
        "fsi_study": fsi,
        "nwt_study": nwt,
        "option_study": opts,
        "roofline": r["roofline"],
        "measured_ceilings": r["ceilings"],
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
