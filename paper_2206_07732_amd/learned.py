"""Harvest, training and evaluation of the learned initial guess.

    python -m paper_2206_07732_amd.learned train --runs 24 --steps 40 --epochs 3 --out weights.npy
    python -m paper_2206_07732_amd.learned eval --weights weights.npy --steps 20

Harvest: seeded 3-D tanks of 128x64x64 cells with Airy waves of amplitude
U[0.01, 0.08] m and period U[0.8, 2] s and the buoy at (x, y) in
U([1.5, 2.5] x [0.75, 1.25]) m are stepped with the FP64 solver; before each
projection the four features and afterwards the target delta* = (p* - p_prev)
/ P0 are kept on the device.  Training: the project's own forward, backward
and Adam kernels, one sample per step, runs split into training and
held-out sets by seed.  Evaluation: CG iterations and projection wall time
to the same 1e-10 residual with a zero, the previous-step and the learned
initial guess on a larger tank.

Every arithmetic step runs in the gfx950 library; this module only draws the
seeded run parameters, moves tensors and sequences library calls.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2206_07732_amd import inputs as I  # noqa: E402

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "guess_c4.npy")


def he_init(n_params_layers, seed: int) -> np.ndarray:
    """He-normal initial weights (std sqrt(2 / fan_in)), zero biases, in the
    library's canonical order (per layer w[co][ci][kz][ky][kx] then b[co]);
    the output layer starts at zero so that the first guess is p_prev."""
    rng = np.random.default_rng(seed)
    out = []
    for q, (ci, co, k) in enumerate(n_params_layers):
        w = rng.standard_normal(co * ci * k ** 3) * math.sqrt(2.0 / (ci * k ** 3))
        out.append(np.zeros_like(w) if q == len(n_params_layers) - 1 else w)
        out.append(np.zeros(co))
    return np.concatenate(out)


LAYERS = [(4, 16, 3), (16, 32, 3), (32, 64, 3), (96, 32, 3), (48, 16, 3), (16, 1, 1)]


def run_workload(seed: int, nx=128, ny=64, nz=64):
    """One seeded harvest tank."""
    a, T, phase, bx, by = I.harvest_draw(seed)
    wl = I.workload("c4train", nx=nx, ny=ny, nz=nz, h=4.0 / nx, seed=seed,
                    wave={"kind": "airy", "a": a, "T": T, "phase": phase},
                    bodies=[I.Body(1, (bx, by, 0.0), (0.25, 0.7, 1.5))])
    return wl


def harvest(seeds, steps: int, log=print):
    """List of (features (4, nz, ny, nx), target (nz, ny, nx), (beta_x, beta_y,
    beta_z)) FP32 device tensors, one per projection solve."""
    import torch

    from paper_2206_07732_amd import ns
    out = []
    for sd in seeds:
        wl = run_workload(sd)
        f = I.make_fields(wl)
        dev = ns.device_fields(f)
        S = ns.Solver(ns.params(wl), dev)
        shp = f["p"].shape
        t = 0.0
        for s in range(steps):
            dt = S.cfl_dt(wl.cfl, wl.dt_max)      # the CFL rule on the current velocity
            S.levelset_advect_reinit(dt)
            S.momentum_step(dt, t + dt)
            pprev = dev["p"].clone()
            feat = torch.empty((4,) + shp, dtype=torch.float32, device="cuda")
            S.features(dt, pprev, feat)
            beta = tuple(S.buffer(k).clone() for k in ("bxf", "byf", "bzf"))
            S.projection_solve(dt)
            tgt = torch.empty(shp, dtype=torch.float32, device="cuda")
            S.target(pprev, tgt)
            if s > 0:                  # the first step starts from p = 0
                out.append((feat, tgt, beta))
            t += dt
        S.close()
        log(f"[harvest] seed {sd}: {steps} steps to t = {t:.3f} s, total samples {len(out)}")
    return out


def train(train_set, val_set, epochs: int, lr: float, seed: int, log=print):
    from paper_2206_07732_amd import ns
    nz, ny, nx = train_set[0][1].shape
    net = ns.Net(nx, ny, nz, training=True)
    net.set_params(he_init(LAYERS, seed))
    hist = []
    rng = np.random.default_rng(seed)

    def val_loss():
        return float(np.mean([net.train_step(f, t, b, 0.0, update=False) for f, t, b in val_set])) \
            if val_set else float("nan")

    v0 = val_loss()
    log(f"[train] initial held-out loss {v0:.4f} (energy-norm ratio; 1.0 = the previous pressure)")
    best, best_v = net.get_params(), v0
    t0 = time.perf_counter()
    for ep in range(epochs):
        order = rng.permutation(len(train_set))
        losses = []
        for q in order:
            f, t, b = train_set[q]
            losses.append(net.train_step(f, t, b, lr))
        v = val_loss()
        if v < best_v:
            best, best_v = net.get_params(), v
        hist.append({"epoch": ep + 1, "train_loss": float(np.mean(losses)), "val_loss": v,
                     "seconds": time.perf_counter() - t0})
        log(f"[train] epoch {ep + 1}: train {np.mean(losses):.4f} held-out {v:.4f} ({time.perf_counter() - t0:.1f}s)")
    log(f"[train] best held-out loss {best_v:.4f}")
    return best, {"initial_val_loss": v0, "best_val_loss": best_v, "epochs": hist}


def evaluate(params, steps: int, wl_name="c3", log=print, precs=("fp64", "mixed")):
    """CG iterations and projection time to 1e-10 for each initial guess."""
    import torch

    from paper_2206_07732_amd import ns
    wl = I.workload(wl_name)
    f = I.make_fields(wl)
    res = {"workload": wl.name, "steps": steps}
    net = None
    if params is not None:
        net = ns.Net(wl.nx, wl.ny, wl.nz)
        net.set_params(params)
    for prec in precs:
        for x0 in ("zero", "prev", "learned"):
            if x0 == "learned" and net is None:
                continue
            dev = ns.device_fields(f)
            S = ns.Solver(ns.params(wl, prec=ns.PREC_FP64 if prec == "fp64" else ns.PREC_MIXED,
                                    x0={"zero": ns.X0_ZERO, "prev": ns.X0_PREV, "learned": ns.X0_LEARNED}[x0]),
                          dev)
            if x0 == "learned":
                S.attach_net(net)
            t, its, ms, r0 = 0.0, [], [], []
            for s in range(steps):
                dt = S.cfl_dt(wl.cfl, wl.dt_max)
                S.levelset_advect_reinit(dt)
                S.momentum_step(dt, t + dt)
                torch.cuda.synchronize()
                a = time.perf_counter()
                st = S.projection_solve(dt)
                ms.append(1e3 * (time.perf_counter() - a))
                its.append(st["iters"])
                r0.append(st["rel_resid0"])
                assert st["true_rel_resid"] <= 1e-10
                t += dt
            key = f"{prec}+{x0}"
            # the first step starts every guess from p = 0: report steps 2..
            res[key] = {"iters": its, "mean_iters": float(np.mean(its[1:])),
                        "median_ms": float(np.median(ms[1:])), "mean_rel_resid0": float(np.mean(r0[1:]))}
            log(f"[eval] {key}: mean iters {np.mean(its[1:]):.2f}, median {np.median(ms[1:]):.3f} ms, "
                f"mean initial rel resid {np.mean(r0[1:]):.3e}")
            S.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    tr = sub.add_parser("train")
    tr.add_argument("--runs", type=int, default=24)
    tr.add_argument("--holdout", type=int, default=3)
    tr.add_argument("--steps", type=int, default=40)
    tr.add_argument("--epochs", type=int, default=3)
    tr.add_argument("--lr", type=float, default=3e-4)
    tr.add_argument("--seed", type=int, default=0)
    tr.add_argument("--out", default=WEIGHTS)
    tr.add_argument("--report", default=None)
    ev = sub.add_parser("eval")
    ev.add_argument("--weights", default=WEIGHTS)
    ev.add_argument("--steps", type=int, default=20)
    ev.add_argument("--workload", default="c3")
    ev.add_argument("--report", default=None)
    a = ap.parse_args()

    def log(*x):
        print(*x, flush=True)

    if a.cmd == "train":
        seeds = list(range(a.runs))
        train_seeds, val_seeds = seeds[:-a.holdout], seeds[-a.holdout:]
        t0 = time.perf_counter()
        train_set = harvest(train_seeds, a.steps, log)
        val_set = harvest(val_seeds, a.steps, log)
        log(f"[harvest] {len(train_set)} training and {len(val_set)} held-out samples "
            f"in {time.perf_counter() - t0:.1f}s")
        params, hist = train(train_set, val_set, a.epochs, a.lr, a.seed, log)
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        np.save(a.out, params.astype(np.float32), allow_pickle=False)
        log(f"[train] wrote {a.out}")
        if a.report:
            json.dump({"train_runs": train_seeds, "holdout_runs": val_seeds, "steps_per_run": a.steps,
                       "samples": len(train_set), "holdout_samples": len(val_set), **hist},
                      open(a.report, "w"), indent=1)
    else:
        params = np.load(a.weights, allow_pickle=False) if a.weights and os.path.exists(a.weights) else None
        res = evaluate(params, a.steps, a.workload, log)
        if a.report:
            json.dump(res, open(a.report, "w"), indent=1)


if __name__ == "__main__":
    main()
