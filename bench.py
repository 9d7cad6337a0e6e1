#!/usr/bin/env python
"""Benchmark of the CROM latent step on one MI355X.

Workload (2D heat on the unit square): decoder (x in R^2, q in R^8) -> 5
ELU layers of width 128 -> 1 with Xavier-uniform weights from a seed;
diffusivity mu ~ U(0.1, 1); 2,000 integration samples uniform in (0, 1)^2;
dt = 1e-4.  One step = the full-field decode of the 65,536 nodes of the
256 x 256 grid plus one latent step q_n -> q_{n+1} at the samples
(decoder with x tangents, Laplacian and latent Jacobian, heat update, and
Gauss-Newton inversion with up to 5 iterations and FP64 normal equations).
The steps form a rollout: each starts from the previous step's latent.

Reported value: decoder+Jacobian point-evals per second, where one
point-eval is one point through the decoder with all 12 columns (value, 2
gradient entries, Laplacian, 8 latent-Jacobian entries; 1,576,448
algorithmic FLOP) and the step's algorithmic decoder work is counted in
that unit.  latent_steps_per_s is reported beside it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec bf16|fp32|bf16x3|bf16pure]
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

W, DEPTH, M, R = 128, 5, 2, 8
FLOP_VALUE_COL = 2 * M * W + 2 * (DEPTH - 1) * W * W + 2 * W        # 131,840
FLOP_TAN_COL = 2 * (DEPTH - 1) * W * W + 2 * W                      # 131,328
FLOP_POINT_EVAL = FLOP_VALUE_COL + (M + 1 + R) * FLOP_TAN_COL      # 1,576,448
TOL_STEP = 1e-6   # Gauss-Newton step tolerance, relative to 1 + |q| (both sides)
PEAK = {"bf16": 2500.0, "bf16x3": 2500.0, "bf16pure": 2500.0, "fp32": 157.3}  # TFLOP/s, dense


def step_flops(S: int, iters: int, ls_evals: int) -> float:
    """Algorithmic decoder FLOP of one latent step: the 12-column evaluation
    at q_n, then per Gauss-Newton iteration the r latent tangents at the new
    iterate, plus one difference column per line-search trial examined."""
    return S * (FLOP_POINT_EVAL + (ls_evals + iters * R) * FLOP_TAN_COL)


def cpu_baseline(wl, nodes, n_steps: int):
    """The FP64 oracle on the host: full-field decode plus latent steps."""
    from oracle import mlp, step as ostep
    from oracle.inversion import GNOptions
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = 1
    dec = mlp.MLPDecoder(wl.layers, wl.m)
    q = wl.q0.copy()
    flop = 0.0
    t0 = time.perf_counter()
    for _ in range(n_steps):
        mlp.decode(wl.layers, nodes, q)
        q, info, _ = ostep.heat_step(dec, wl.samples, q, wl.mu, wl.dt,
                                     GNOptions(max_iter=5, tol_step=TOL_STEP))
        flop += len(nodes) * FLOP_VALUE_COL + step_flops(len(wl.samples), info.iters, info.ls_evals)
    dt = time.perf_counter() - t0
    return {"value": flop / FLOP_POINT_EVAL / dt, "unit": "point-evals/s", "cores": cores,
            "kind": "oracle", "sample": f"{n_steps} steps (full-field decode of {len(nodes)} nodes + "
            f"one Gauss-Newton latent step at {len(wl.samples)} samples each), FP64 NumPy, {dt:.1f} s",
            "latent_steps_per_s": n_steps / dt}


def batched_leg(args, crom, torch, dev):
    """Batched rollout: 512 instances of 2D heat, mu_i ~ U(0.1, 1), sample
    counts S_i ~ U{200..2000} drawn without replacement from the interior
    nodes of a 128 x 128 lattice, r = 8, dt = 1e-4; all instances advance
    together in one step launch.  Gauss-Newton (5 iterations, tol 1e-6) and
    the linearised inversion are timed separately."""
    from workloads import Batched2D
    wb = Batched2D(seed=args.seed)
    dec = crom.Decoder.from_layers(wb.layers, wb.m, precision=args.prec, device=dev)
    st = crom.Stepper(dec, wb.offsets, torch.from_numpy(wb.samples).to(dev))
    nu = torch.from_numpy(wb.mu).to(dev)
    out = {"workload": f"{wb.n_inst} instances, S_i in [{wb.s_min},{wb.s_max}], total samples "
                       f"{int(wb.offsets[-1])}", "steps": args.batched_steps}
    total = int(wb.offsets[-1])
    for name, opts in (("gn", crom.GNOptions(max_iter=5, tol_step=TOL_STEP)),
                       ("lls", crom.GNOptions(max_iter=1, linearized=True))):
        q = [torch.from_numpy(wb.q0.copy()).to(dev), torch.empty(wb.n_inst, R, dtype=torch.float64, device=dev)]
        for i in range(3):
            st.step(q[i % 2], nu, wb.dt, opts, q_next=q[(i + 1) % 2])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        flop = 0.0
        infos = []
        e0.record()
        for i in range(args.batched_steps):
            st.step(q[i % 2], nu, wb.dt, opts, q_next=q[(i + 1) % 2])
        e1.record()
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) * 1e-3 / args.batched_steps
        inf = st.info()  # iteration counts of the last step stand for all
        flop = sum(step_flops(int(wb.offsets[k + 1] - wb.offsets[k]), int(inf["iters"][k]),
                              int(inf["ls_evals"][k])) for k in range(wb.n_inst))
        if opts.linearized:
            flop = total * (FLOP_POINT_EVAL)
        achieved = flop / t / 1e12
        out[name] = {"ms_per_step": t * 1e3, "instance_steps_per_s": wb.n_inst / t,
                     "point_evals_per_s": flop / FLOP_POINT_EVAL / t,
                     "achieved_tflops": achieved, "frac_of_peak": achieved / PEAK[args.prec],
                     "gn_iters_mean": float(inf["iters"].mean()), "ls_evals_mean": float(inf["ls_evals"].mean())}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--prec", default="bf16", choices=sorted(PEAK))
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--batched-steps", type=int, default=20)
    args = ap.parse_args()
    if args.gpus != 1:
        print("this benchmark runs on one GPU: the instances of a batch are independent and the "
              "step of one instance is not split across devices", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2206_02607_amd import crom
    from workloads import Heat2D

    dev = torch.device("cuda:0")
    wl = Heat2D(seed=args.seed)
    nodes = wl.nodes
    dec = crom.Decoder.from_layers(wl.layers, wl.m, precision=args.prec, device=dev)
    X = torch.from_numpy(nodes).to(dev)
    st = crom.Stepper(dec, [0, wl.n_samples], torch.from_numpy(wl.samples).to(dev))
    q = [torch.from_numpy(wl.q0[None].copy()).to(dev), torch.empty(1, R, dtype=torch.float64, device=dev)]
    nu = torch.tensor([wl.mu], dtype=torch.float64, device=dev)
    g = torch.empty(len(nodes), 1, dtype=torch.float32, device=dev)
    opts = crom.GNOptions(max_iter=5, tol_step=TOL_STEP)

    def one(i, ev=None):
        if ev is not None:
            ev[0].record()
        dec.decode(X, q[i % 2], out=g)
        if ev is not None:
            ev[1].record()
        st.step(q[i % 2], nu, wl.dt, opts, q_next=q[(i + 1) % 2])
        if ev is not None:
            ev[2].record()

    for i in range(args.warmup):
        one(i)
    torch.cuda.synchronize()
    infos = []
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        one(args.warmup + i, evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # per-step work: the step's iteration counts (one sync per step, outside the timed region)
    t_dec = np.array([e[0].elapsed_time(e[1]) for e in evs]) * 1e-3
    t_step = np.array([e[1].elapsed_time(e[2]) for e in evs]) * 1e-3
    # iteration statistics of the timed rollout: rerun it untimed, step by step
    q[0].copy_(torch.from_numpy(wl.q0[None].copy()))
    for i in range(args.warmup):
        one(i)
    flop_step = 0.0
    for i in range(args.steps):
        one(args.warmup + i)
        inf = st.info()[0]
        infos.append(inf)
        flop_step += step_flops(wl.n_samples, int(inf["iters"]), int(inf["ls_evals"]))
    torch.cuda.synchronize()
    flop_dec = args.steps * len(nodes) * FLOP_VALUE_COL
    value = (flop_dec + flop_step) / FLOP_POINT_EVAL / wall
    ms = wall / args.steps * 1e3

    # dominant kernel for the roofline
    dec_flop = len(nodes) * FLOP_VALUE_COL
    cand = {"decode": (t_dec.mean(), dec_flop), "step": (t_step.mean(), flop_step / args.steps)}
    name = max(cand, key=lambda k: cand[k][0])
    t_avg, fl = cand[name]
    achieved = fl / t_avg / 1e12
    roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK[args.prec], "unit": "TFLOP/s",
            "frac": achieved / PEAK[args.prec], "traffic": None,
            "kernel": {"decode": "decode_kernel (full field, value column)",
                       "step": "step_kernel (cooperative latent step)"}[name],
            "avg_ms": t_avg * 1e3, "flop_per_launch": fl,
            "other": {k: {"avg_ms": v[0] * 1e3, "achieved_tflops": v[1] / v[0] / 1e12}
                      for k, v in cand.items() if k != name}}

    # the linearised inversion (one normal-equation solve per step), same rollout
    lls = crom.GNOptions(max_iter=1, linearized=True)
    q[0].copy_(torch.from_numpy(wl.q0[None].copy()))
    for i in range(args.warmup):
        st.step(q[i % 2], nu, wl.dt, lls, q_next=q[(i + 1) % 2])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for i in range(args.steps):
        st.step(q[i % 2], nu, wl.dt, lls, q_next=q[(i + 1) % 2])
    torch.cuda.synchronize()
    lls_steps_per_s = args.steps / (time.perf_counter() - t1)

    batched = batched_leg(args, crom, torch, dev) if args.batched_steps > 0 else None
    cpu = cpu_baseline(wl, nodes, args.cpu_steps) if args.cpu_steps > 0 else None
    its = np.array([int(i["iters"]) for i in infos])
    lse = np.array([int(i["ls_evals"]) for i in infos])
    out = {
        "metric": "decoder+Jacobian point-evals/sec and latent steps/sec at fixed rollout error",
        "value": value, "unit": "point-evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.prec, "data": "synthetic",
        "config": {"workload": "2D heat, 256x256 grid: full-field decode of 65,536 nodes + one "
                               "Gauss-Newton latent step at 2,000 samples per step",
                   "decoder": "(x in R^2, q in R^8) -> 5 x ELU width 128 -> 1, Xavier-uniform, seed "
                              f"{args.seed}",
                   "mu": wl.mu, "dt": wl.dt, "gn_max_iter": 5, "precision": args.prec},
        "latent_steps_per_s": args.steps / wall,
        "lls_latent_steps_per_s": lls_steps_per_s,
        "gn_tol_step": TOL_STEP,
        "step_ms_avg": t_step.mean() * 1e3, "decode_ms_avg": t_dec.mean() * 1e3,
        "gn_iters_mean": float(its.mean()), "ls_evals_mean": float(lse.mean()),
        "roofline": roof,
        "batched": batched,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
