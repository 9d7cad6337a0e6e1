#!/usr/bin/env python
"""Benchmark of the CROM latent step on one MI355X.

Headline workload: the batched rollout of 512 instances of 2D heat on the
unit square (mu_i ~ U(0.1, 1), S_i ~ U{200..2000} integration samples drawn
from the interior nodes of a 128 x 128 lattice, dt = 1e-4) with the decoder
(x in R^2, q in R^8) -> 5 ELU layers of width 128 -> 1 trained by the
library's own kernels on FP64 finite-difference snapshots (the training
leg runs first).  One step = one latent step q_n -> q_{n+1} of every
instance: the decoder with x tangents, Laplacian and latent Jacobian at the
samples, the heat update and the inversion (FP64 normal equations).  Four
modes (Gauss-Newton or linearised inversion, BF16 or FP32 decoder
arithmetic) are timed; each one's rollout error over 500 steps is judged by
the FP64 finite-difference solver on a subset, and the headline is the
fastest mode at the best mode's rollout error.

Reported value: decoder+Jacobian point-evals per second, one point-eval
being one point through the decoder with value, 2 gradient entries,
Laplacian and the 8 latent-Jacobian entries; latent steps per second
(instance-steps) beside it.  The step forms the latent Jacobian by a
reverse (adjoint) pass: 658,944 algorithmic FLOP per point-eval (value,
x tangents and Laplacian forward, one adjoint column back); a Gauss-Newton
step's further iterations and trials are counted in units of that
evaluation.  roofline:
the headline mode's timed kernels against the matrix-core peak of its
arithmetic; cpu_baseline: the FP64 oracle on a bounded sample of the same
workload.

Further legs: the single-instance 2D heat step at 2,000 samples with a
full-field decode (latency-bound), the 1D and 3D workloads, the training
step, sample selection, the encoder guess, SIREN and corotated FE.

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
# the linearised step's evaluation: value, x tangents and Laplacian forward,
# the latent Jacobian by one adjoint column back through the hidden layers
# and the first layer's latent columns
FLOP_ADJ_COL = 2 * (DEPTH - 1) * W * W + 2 * W * R                  # 133,120
FLOP_POINT_EVAL_LLS = FLOP_VALUE_COL + (M + 1) * FLOP_TAN_COL + FLOP_ADJ_COL  # 658,944
# Gauss-Newton step tolerance, relative to 1 + |q|.  The same 1e-6 for every
# arithmetic: the change of q over one time step is about 1e-4 of |q| here,
# and the stopping rule stops without moving when the Gauss-Newton step is
# below tol (1 + |q|), so a coarser tolerance (1e-3) would freeze the
# rollout.  Steps that reach the 5-iteration cap report MAXITER (not a
# failure); the flags of every timed leg are reported.
TOL_STEP = {"bf16": 1e-6, "bf16pure": 1e-6, "bf16x3": 1e-6, "fp32": 1e-6}
PEAK = {"bf16": 2500.0, "bf16x3": 2500.0, "bf16pure": 2500.0, "fp32": 157.3}  # TFLOP/s, dense
# flags of a failed instance-step (its work does not count as throughput)
FAILED = 2 | 4 | 8 | 16  # SINGULAR | NONFINITE | LS_FAIL | ABORTED


def source_hash() -> str:
    """sha256 of the sources the step and decode kernels are built from (a
    hardware-counter measurement holds only for the build it was taken on)."""
    import hashlib
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_2206_02607_amd", "csrc")
    for name in ("common.hpp", "engine.hpp", "tune.hpp", "decode.hip", "step.hip", "../../include/crom.h"):
        path = os.path.normpath(os.path.join(src, name))
        with open(path, "rb") as f:
            h.update(os.path.basename(path).encode() + f.read())
    return h.hexdigest()


def measured_traffic(kernel: str, summary: str = "traffic_2d_heat.json"):
    """HBM bytes per launch of `kernel` from a committed counter summary,
    when it was taken on the current sources; else None."""
    path = os.path.join(ROOT, "profiles", summary)
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != source_hash():
        return None
    k = t.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def step_flops(S: int, iters: int, ls_evals: int) -> float:
    """Algorithmic decoder FLOP of one Gauss-Newton latent step as the
    library forms it for these depths (the reverse pass): the evaluation at
    q_n (value, x tangents and Laplacian forward, the latent Jacobian by one
    adjoint column), then per iteration the adjoint column at the new
    iterate, and one difference column per line-search trial examined."""
    return S * (FLOP_POINT_EVAL_LLS + iters * FLOP_ADJ_COL + ls_evals * FLOP_TAN_COL)


def _cores():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        return 1


def cpu_baseline_batched(wb, opts_kw: dict, budget_s: float):
    """The FP64 oracle on the host, on a bounded sample of the batched
    workload: one latent step of the batch's instances 0, 1, 2, ... in turn
    (the workload's own seeded weights and latents: the same arithmetic per
    sample as any trained network) until about budget_s seconds have been
    spent, counted in the headline's unit."""
    from oracle import mlp, step as ostep
    from oracle.inversion import GNOptions
    dec = mlp.MLPDecoder(wb.layers, wb.m)
    flop, n, S_tot = 0.0, 0, 0
    t0 = time.perf_counter()
    while n < wb.n_inst and (n == 0 or time.perf_counter() - t0 < budget_s):
        y = wb.samples[wb.offsets[n]:wb.offsets[n + 1]]
        _, info, _ = ostep.heat_step(dec, y, wb.q0[n], float(wb.mu[n]), wb.dt, GNOptions(**opts_kw))
        S = len(y)
        flop += S * FLOP_POINT_EVAL_LLS if opts_kw.get("linearized") else step_flops(S, info.iters, info.ls_evals)
        S_tot += S
        n += 1
    dt = time.perf_counter() - t0
    return {"value": flop / FLOP_POINT_EVAL_LLS / dt, "unit": "point-evals/s", "cores": _cores(), "kind": "oracle",
            "sample": f"one latent step ({'linearised' if opts_kw.get('linearized') else 'Gauss-Newton'}) of "
                      f"instances 0..{n - 1} of the 512-instance batch ({S_tot} samples), FP64 NumPy, {dt:.1f} s",
            "latent_steps_per_s": n / dt}


def cpu_baseline(wl, nodes, n_steps: int):
    """The FP64 oracle on the host: full-field decode plus latent steps."""
    from oracle import mlp, step as ostep
    from oracle.inversion import GNOptions
    cores = _cores()
    dec = mlp.MLPDecoder(wl.layers, wl.m)
    q = wl.q0.copy()
    flop = 0.0
    t0 = time.perf_counter()
    for _ in range(n_steps):
        mlp.decode(wl.layers, nodes, q)
        q, info, _ = ostep.heat_step(dec, wl.samples, q, wl.mu, wl.dt,
                                     GNOptions(max_iter=5, tol_step=TOL_STEP["fp32"]))
        flop += len(nodes) * FLOP_VALUE_COL + step_flops(len(wl.samples), info.iters, info.ls_evals)
    dt = time.perf_counter() - t0
    return {"value": flop / FLOP_POINT_EVAL_LLS / dt, "unit": "point-evals/s", "cores": cores,
            "kind": "oracle", "sample": f"{n_steps} steps (full-field decode of {len(nodes)} nodes + "
            f"one Gauss-Newton latent step at {len(wl.samples)} samples each), FP64 NumPy, {dt:.1f} s",
            "latent_steps_per_s": n_steps / dt}


def train_flops(B: int, P: int, m: int, r: int, d: int, width: int, depth: int, n_in: int, hidden: int) -> float:
    """Algorithmic FLOP of one training step (forward, backward; Adam and the
    loss are O(parameters) and O(B P) and left out): every multiply-add of the
    decoder at B * P points and of the encoder on B snapshots, counted once."""
    rows = B * P
    hid = (depth - 1) * width * width
    dec_fwd = rows * (m * width + hid + width * d) + B * r * width
    dec_bwd = rows * (2 * width * d + 2 * hid + m * width) + B * r * width
    enc = B * (n_in * hidden + hidden * r) + B * (hidden * r + r * hidden + n_in * hidden)
    return 2.0 * (dec_fwd + dec_bwd + enc)


def train_leg(args, crom, torch, dev):
    """Decoder training (16 x 16,384-point batches of 2D heat snapshots from
    the FP64 finite-difference solver; encoder 16,384 -> 256 -> 8): the
    training step timed in BF16 and FP32, then a BF16 training run of
    --train-steps steps whose network the batched leg uses."""
    from paper_2206_02607_amd import heat2d
    from workloads import Train2D
    w = Train2D(seed=args.seed)
    u0 = w.initial_field()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    e[0].record()
    snaps = heat2d.fd_snapshots(u0, w.mu, w.times, w.dx, w.dt_fd, dev)
    e[1].record()
    torch.cuda.synchronize()
    rows = snaps.reshape(-1, w.grid * w.grid)
    nodes = torch.from_numpy(w.nodes).to(dev)
    sd = heat2d.Standardization.of(rows, nodes)
    data, xs = sd.data(rows), sd.points(nodes)
    enc0 = np.concatenate([np.concatenate([Wm.ravel(), b.ravel()]) for Wm, b in w.enc_layers]).astype(np.float32)
    P = w.grid * w.grid
    fl = train_flops(w.batch, P, w.m, w.r, w.d, w.width, w.depth, P * w.d, w.enc_hidden)
    out = {"workload": f"{w.n_mu} diffusivities x {len(w.times)} times = {rows.shape[0]} FP64 snapshots of "
                       f"{w.grid}x{w.grid} nodes; batch {w.batch} snapshots ({w.batch * P} decoder points); "
                       f"encoder {P}->{w.enc_hidden}->{w.r}",
           "fd_snapshots_ms": e[0].elapsed_time(e[1]), "flop_per_step": fl}

    def make(prec):
        dec = crom.Decoder.from_layers(w.layers, w.m, precision=prec, device=dev)
        return dec, crom.Trainer(dec, enc0.copy(), w.enc_hidden, xs, w.batch)

    for prec in args.train_precs.split(","):
        dec, T = make(prec)
        for _ in range(3):
            T.step(data[:w.batch], 1e-4)
        torch.cuda.synchronize()
        e[0].record()
        for k in range(args.train_time_steps):
            T.step(data[(k % 12) * w.batch:(k % 12 + 1) * w.batch], 1e-4)
        e[1].record()
        torch.cuda.synchronize()
        t = e[0].elapsed_time(e[1]) * 1e-3 / args.train_time_steps
        out[prec] = {"ms_per_step": t * 1e3, "steps_per_s": 1.0 / t, "achieved_tflops": fl / t / 1e12,
                     "frac_of_peak": fl / t / 1e12 / PEAK[prec]}
    if args.train_conv:
        # the paper's convolutional encoder (16,384 -> 4095 -> 1023 -> 255 -> 63,
        # dense 32, r), seeded uniform parameters: the step time with it
        from workloads import rng as _rng
        n_conv = crom.encoder_param_count(P * w.d, 32, w.r, "conv", w.d)
        enc_conv = _rng(args.seed + 5).uniform(-0.1, 0.1, size=n_conv).astype(np.float32)
        decc = crom.Decoder.from_layers(w.layers, w.m, precision="bf16", device=dev)
        Tc = crom.Trainer(decc, enc_conv, 32, xs, w.batch, enc_kind="conv")
        for _ in range(3):
            Tc.step(data[:w.batch], 1e-4)
        torch.cuda.synchronize()
        e[0].record()
        for k in range(args.train_time_steps):
            Tc.step(data[(k % 12) * w.batch:(k % 12 + 1) * w.batch], 1e-4)
        e[1].record()
        torch.cuda.synchronize()
        out["bf16_conv_encoder"] = {"ms_per_step": e[0].elapsed_time(e[1]) / args.train_time_steps,
                                    "encoder_params": n_conv}
    if args.train_steps <= 0:
        return out, None
    dec, T = make("bf16")
    t0 = time.perf_counter()
    losses = heat2d.train(T, data, args.train_steps, seed=1)
    torch.cuda.synchronize()
    out["run"] = {"steps": args.train_steps, "seconds": time.perf_counter() - t0,
                  "loss_first50": float(losses[:50].mean()), "loss_last50": float(losses[-50:].mean()),
                  "schedule": "lr = 1e-4 x (10, 5, 2, 1, 0.5, 0.2) in equal stages, standardized data"}
    sd.fold(dec, T.enc_params, T.n_in, T.hidden)
    q0 = T.encode(torch.from_numpy(u0.astype(np.float32)).to(dev).reshape(1, -1)).cpu().numpy()[0]
    err0 = heat2d.rel_error(heat2d.decode_fields(dec, nodes, q0[None].astype(np.float64)),
                            torch.from_numpy(u0).to(dev).reshape(1, -1))[0]
    out["run"]["initial_field_error"] = float(err0)
    return out, {"params": dec.params.detach().clone(), "q0": q0.astype(np.float64), "w": w, "u0": u0,
                 "nodes": nodes, "enc": T.enc_params.detach().clone(), "hidden": T.hidden}


def batched_leg(args, crom, torch, dev, trained=None):
    """The headline: batched rollout of 512 instances of 2D heat, mu_i ~
    U(0.1, 1), sample counts S_i ~ U{200..2000} drawn without replacement
    from the interior nodes of a 128 x 128 lattice, r = 8, dt = 1e-4, with
    the trained network (the training leg's; every instance starts from the
    encoded initial field).  All instances advance together in one step.

    Four modes: Gauss-Newton (5 iterations, step tolerance per arithmetic)
    and the linearised inversion, each with BF16 and FP32 decoder arithmetic.
    For each: the rollout error of the first --judge instances over 500 steps
    against the FP64 finite-difference solution (space-time relative L2 at 5
    recorded states), then K timed steps of the whole batch after W warm-up
    steps, and the same K steps replayed untimed with the per-instance
    outcome read after every step (iterations, line-search trials, flags).
    Failed instance-steps (SINGULAR, NONFINITE, LS_FAIL, ABORTED) do not
    count as work.  The headline mode is the fastest one whose rollout error
    equals the best mode's (at most 1.05 times it, or within 1e-4)."""
    from paper_2206_02607_amd import heat2d
    from workloads import Batched2D
    wb = Batched2D(seed=args.seed)
    params = trained["params"] if trained else crom.flatten_layers(wb.layers)
    q_init = np.tile(trained["q0"], (wb.n_inst, 1)) if trained else wb.q0
    total = int(wb.offsets[-1])
    S = np.diff(wb.offsets)
    out = {"workload": f"{wb.n_inst} instances of 2D heat, S_i in [{wb.s_min},{wb.s_max}] samples of the "
                       f"{wb.grid}x{wb.grid} lattice (total {total}), r = 8, dt = {wb.dt}",
           "net": "trained (training leg), (x in R^2, q in R^8) -> 5 x ELU width 128 -> 1" if trained
                  else "Xavier-uniform, untrained"}
    nu = torch.from_numpy(wb.mu).to(dev)
    record = [0, 125, 250, 375, 500]
    nj = min(args.judge, wb.n_inst) if trained else 0
    if nj:
        w = trained["w"]
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        e[0].record()
        ref = heat2d.fd_snapshots(trained["u0"], wb.mu[:nj], [k * wb.dt for k in record], w.dx, w.dt_fd, dev)
        e[1].record()
        torch.cuda.synchronize()
        refs = [ref[:, k].reshape(nj, -1) for k in range(len(record))]
        out["fd_judge"] = {"instances": nj, "ms": e[0].elapsed_time(e[1]),
                           "substeps": int(round(record[-1] * wb.dt / w.dt_fd))}
    precs = (args.prec, "fp32") if args.prec != "fp32" else ("fp32",)
    modes = {}
    for prec in precs:
        dec = crom.Decoder(params, wb.m, wb.r, wb.d, wb.width, wb.depth, prec, dev)
        st = crom.Stepper(dec, wb.offsets, torch.from_numpy(wb.samples).to(dev))
        for kind, opts in (("lls", crom.GNOptions(max_iter=1, linearized=True)),
                           ("gn", crom.GNOptions(max_iter=5, tol_step=TOL_STEP[prec]))):
            if args.modes and f"{prec}_{kind}" not in args.modes.split(","):
                continue
            r = {"precision": prec, "inversion": "linearised" if opts.linearized else "Gauss-Newton",
                 "tol_step": None if opts.linearized else TOL_STEP[prec]}
            if nj:
                ro = heat2d.rollout(dec, np.tile(trained["q0"], (nj, 1)), wb.samples[:int(wb.offsets[nj])],
                                    wb.mu[:nj], wb.dt, record[-1], opts, record, offsets=wb.offsets[:nj + 1])
                fields = [heat2d.decode_fields(dec, trained["nodes"], qq) for qq in ro.q]
                err = heat2d.spacetime_error(fields, refs)
                r["rollout_error_mean"] = float(err.mean())
                r["rollout_error_max"] = float(err.max())
                r["rollout_flags_or"] = int(np.bitwise_or.reduce(ro.flags[-1]))
            q = [torch.from_numpy(np.asarray(q_init, np.float64).copy()).to(dev),
                 torch.empty(wb.n_inst, R, dtype=torch.float64, device=dev)]
            for i in range(args.warmup):
                st.step(q[i % 2], nu, wb.dt, opts, q_next=q[(i + 1) % 2])
            q_w = q[args.warmup % 2].clone()
            torch.cuda.synchronize()
            crom.kernel_timer(True)
            t0 = time.perf_counter()
            for i in range(args.steps):
                st.step(q[(args.warmup + i) % 2], nu, wb.dt, opts, q_next=q[(args.warmup + i + 1) % 2])
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            crom.kernel_timer(False)
            k_ms, k_n = crom.kernel_timer_read()
            # the same steps again, untimed, reading every step's outcome
            q[args.warmup % 2].copy_(q_w)
            flop, pevals, n_fail, flags_or, iters, lse = 0.0, 0.0, 0, 0, 0, 0
            for i in range(args.steps):
                st.step(q[(args.warmup + i) % 2], nu, wb.dt, opts, q_next=q[(args.warmup + i + 1) % 2])
                inf = st.info()
                ok = (inf["flags"] & FAILED) == 0
                n_fail += int((~ok).sum())
                flags_or |= int(np.bitwise_or.reduce(inf["flags"]))
                iters += int(inf["iters"].sum())
                lse += int(inf["ls_evals"].sum())
                if opts.linearized:
                    pevals += float(S[ok].sum())
                    flop += float(S[ok].sum()) * FLOP_POINT_EVAL_LLS
                else:
                    f = sum(step_flops(int(S[k]), int(inf["iters"][k]), int(inf["ls_evals"][k]))
                            for k in np.flatnonzero(ok))
                    flop += f
                    pevals += f / FLOP_POINT_EVAL_LLS
            t = wall / args.steps
            kernel_ms = k_ms / max(1, k_n)
            fl_step = flop / args.steps
            r.update({"ms_per_step": t * 1e3, "instance_steps_per_s": (wb.n_inst * args.steps - n_fail) / wall,
                      "point_evals_per_s": pevals / wall,
                      "achieved_tflops": fl_step / t / 1e12, "frac_of_peak": fl_step / t / 1e12 / PEAK[prec],
                      "timed_kernels": ("lls_jets_kernel (forward value, x tangents and Laplacian, reverse "
                                        "latent Jacobian)" if opts.linearized else
                                        "gn_round_kernel + gn_solve_kernel, every round of the step"),
                      "timed_kernels_ms": kernel_ms, "flop_per_step": fl_step,
                      "gn_iters_mean": iters / (wb.n_inst * args.steps),
                      "ls_evals_mean": lse / (wb.n_inst * args.steps),
                      "failed_instance_steps": n_fail, "flags_or": flags_or})
            modes[f"{prec}_{kind}"] = r
    out["modes"] = modes
    if not modes:
        raise SystemExit(f"--modes {args.modes!r} selects none of the batched modes of precisions {precs}")
    errs = {k: v.get("rollout_error_mean") for k, v in modes.items()}
    if all(e is not None for e in errs.values()):
        best = min(errs.values())
        equal = [k for k, e in errs.items() if e <= max(1.05 * best, best + 1e-4)]
        rule = "fastest mode whose rollout error is at most 1.05x the best mode's (or within 1e-4)"
    else:
        equal = list(modes)
        rule = "no rollout error measured (untrained network): fastest mode"
    head = max(equal, key=lambda k: modes[k]["point_evals_per_s"])
    out["headline_mode"] = head
    out["headline_rule"] = rule
    if len(precs) == 2 and len(modes) == 4:
        a, b = precs
        out["precision_study"] = {
            kind: {"speedup_" + a + "_vs_fp32": modes[f"{b}_{kind}"]["ms_per_step"] / modes[f"{a}_{kind}"]["ms_per_step"],
                   "rollout_error_" + a: modes[f"{a}_{kind}"].get("rollout_error_mean"),
                   "rollout_error_fp32": modes[f"{b}_{kind}"].get("rollout_error_mean")}
            for kind in ("gn", "lls")}
    return out


def sampling_leg(args, crom, torch, dev, trained):
    """Robust greedy sample selection (Appendix "Robust Sampling") with the
    trained network: the residual vector sums, over every training
    diffusivity, the final-time (500 linearised steps) error at all 16,384
    nodes against the FP64 finite-difference solution; 10 candidates per
    round, from 8 random interior nodes.  Reports seconds per round, the
    metric before and after, the metric of random sets of the final size,
    and the fused residual kernel's throughput on one round's 10 x n_mu
    final latents."""
    from paper_2206_02607_amd import heat2d
    w, u0, nodes = trained["w"], trained["u0"], trained["nodes"]
    dec = crom.Decoder(trained["params"], w.m, w.r, w.d, w.width, w.depth, args.prec, dev)
    n_mu, P = w.n_mu, w.grid * w.grid
    n_steps = int(round(w.times[-1] / w.dt))
    ref = heat2d.fd_snapshots(u0, w.mu, [w.times[-1]], w.dx, w.dt_fd, dev)[:, 0].reshape(n_mu, P, 1).contiguous()
    gi = np.arange(w.grid)
    edge = (gi == 0) | (gi == w.grid - 1)
    clamp_np = (edge[:, None] | edge[None, :]).reshape(-1).astype(np.uint8)
    clamp = torch.from_numpy(clamp_np).to(dev)
    interior = np.flatnonzero(clamp_np == 0)
    g = np.random.Generator(np.random.PCG64(args.seed + 7))
    q0 = np.tile(trained["q0"], (n_mu, 1))
    opts = crom.GNOptions(max_iter=1, linearized=True)
    init = g.choice(interior, w.r, replace=False)
    n_final = w.r + args.sampling_rounds
    args_ = (dec, nodes, ref, q0, w.mu, w.dt)
    first = crom.robust_sampling(*args_, init, n_steps, 0.0, max_samples=w.r, opts=opts, node_clamp=clamp)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = crom.robust_sampling(*args_, init, n_steps, 0.0, n_try=10, max_samples=n_final, opts=opts,
                               node_clamp=clamp)
    sec = time.perf_counter() - t0
    rand = [crom.robust_sampling(*args_, g.choice(interior, n_final, replace=False), n_steps, 0.0,
                                 max_samples=n_final, opts=opts, node_clamp=clamp).metric for _ in range(3)]
    # the residual kernel alone on 10 x n_mu latents near the trained initial latent
    qs = torch.from_numpy(q0[None].repeat(10, 0) + 0.01 * g.standard_normal((10, n_mu, w.r))).to(dev)
    crom.sampling_residual(dec, nodes, qs, ref)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record()
    for _ in range(reps):
        crom.sampling_residual(dec, nodes, qs, ref)
    e1.record()
    torch.cuda.synchronize()
    t_res = e0.elapsed_time(e1) * 1e-3 / reps
    flop_res = 10 * n_mu * P * FLOP_VALUE_COL
    return {"workload": f"{n_mu} training diffusivities, {P} nodes, {n_steps} linearised steps per rollout, "
                        f"10 candidates per round, {w.r} -> {n_final} samples",
            "rounds": out.rounds, "seconds": sec, "seconds_per_round": sec / max(1, out.rounds),
            "rollout_instance_steps_per_round": 10 * n_mu * n_steps,
            "metric_initial": first.metric, "metric_final": out.metric,
            "metric_random_sets": rand, "samples": out.samples.tolist(),
            "residual_kernel": {"ms": t_res * 1e3, "latents": 10 * n_mu, "nodes": P,
                                "achieved_tflops": flop_res / t_res / 1e12,
                                "frac_of_peak": flop_res / t_res / 1e12 / PEAK[args.prec]}}


def siren_leg(args, crom, torch, dev):
    """The sine-activated decoder (SIREN, omega_0 = 30 folded into the
    weights) of the 2D shape, inputs in [-1, 1]^2: full-field value decode of
    the 256 x 256 grid, the 12-column decode at the same nodes, and the
    single-instance Gauss-Newton heat step at 2,000 samples, in BF16 and
    FP32, and (BF16) one training step of the 2D training workload with the
    SIREN decoder (the ELU numbers of the same shapes are the main line's)."""
    from workloads import Heat2D, rng, siren_mlp
    wl = Heat2D(seed=args.seed)
    layers = siren_mlp(rng(args.seed + 11), wl.m, wl.r, wl.d, wl.width, wl.depth)
    nodes = torch.from_numpy((2.0 * wl.nodes - 1.0).astype(np.float32)).to(dev)
    samples = torch.from_numpy((2.0 * wl.samples - 1.0).astype(np.float32)).to(dev)
    q0 = torch.from_numpy(wl.q0).to(dev)
    P = nodes.shape[0]
    out = {"net": "SIREN (2 + 8) -> 5 x sine width 128 -> 1, omega_0 = 30, seeded SIREN initialisation"}
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for prec in (args.prec, "fp32"):
        dec = crom.Decoder.from_layers(layers, wl.m, precision=prec, device=dev, act="sine")
        g = torch.empty(P, 1, dtype=torch.float32, device=dev)
        for _ in range(3):
            dec.decode(nodes, q0, out=g)
        e[0].record()
        for _ in range(20):
            dec.decode(nodes, q0, out=g)
        e[1].record()
        torch.cuda.synchronize()
        t_val = e[0].elapsed_time(e[1]) * 1e-3 / 20
        for _ in range(2):
            dec.decode_jac(nodes, q0, dx=True, d2=crom.D2_LAPLACIAN, dq=True)
        e[0].record()
        for _ in range(10):
            dec.decode_jac(nodes, q0, dx=True, d2=crom.D2_LAPLACIAN, dq=True)
        e[1].record()
        torch.cuda.synchronize()
        t_jac = e[0].elapsed_time(e[1]) * 1e-3 / 10
        st = crom.Stepper(dec, [0, wl.n_samples], samples)
        nu = torch.tensor([wl.mu], dtype=torch.float64, device=dev)
        opts = crom.GNOptions(max_iter=5, tol_step=TOL_STEP[prec])
        q = [q0[None].clone(), torch.empty(1, R, dtype=torch.float64, device=dev)]
        for i in range(5):
            st.step(q[i % 2], nu, wl.dt, opts, q_next=q[(i + 1) % 2])
        torch.cuda.synchronize()
        crom.kernel_timer(True)
        e[0].record()
        n_steps = 50
        for i in range(n_steps):
            st.step(q[i % 2], nu, wl.dt, opts, q_next=q[(i + 1) % 2])
        e[1].record()
        torch.cuda.synchronize()
        crom.kernel_timer(False)
        k_ms, k_n = crom.kernel_timer_read()
        inf = st.info()[0]
        gn_ms = e[0].elapsed_time(e[1]) / n_steps
        train_ms = None
        if prec != "fp32":  # the sine training path runs on the bfloat16 row kernels
            from workloads import Train2D
            w2 = Train2D(seed=args.seed)
            xs = torch.from_numpy((2.0 * w2.nodes - 1.0).astype(np.float32)).to(dev)
            enc0 = np.concatenate([np.concatenate([Wm.ravel(), b.ravel()]) for Wm, b in w2.enc_layers]).astype(np.float32)
            tdec = crom.Decoder.from_layers(layers, wl.m, precision=prec, device=dev, act="sine")
            T = crom.Trainer(tdec, enc0, w2.enc_hidden, xs, w2.batch)
            ub = torch.randn(w2.batch, xs.shape[0], device=dev) * 0.5
            for _ in range(3):
                T.step(ub, 1e-4)
            e[0].record()
            for _ in range(20):
                T.step(ub, 1e-4)
            e[1].record()
            torch.cuda.synchronize()
            train_ms = e[0].elapsed_time(e[1]) / 20
        out[prec] = {"value_decode_ms": t_val * 1e3, "value_decode_tflops": P * FLOP_VALUE_COL / t_val / 1e12,
                     "train_step_ms": train_ms,
                     "jac_decode_ms": t_jac * 1e3, "jac_decode_tflops": P * FLOP_POINT_EVAL / t_jac / 1e12,
                     "gn_step_ms": gn_ms, "gn_step_kernel_ms": k_ms / max(1, k_n),
                     "gn_iters_last": int(inf["iters"]), "ls_evals_last": int(inf["ls_evals"]),
                     "flags_last": int(inf["flags"])}
    return out


def config1_leg(args, crom, torch, dev):
    """1D heat (nu = 0.5, decoder (1 + 3) -> 5 x 32 -> 1, 20 samples, dt =
    1e-5): a 1000-step Gauss-Newton rollout in FP32 on the GPU, the same
    rollout by the FP64 oracle on one host thread, and their difference."""
    from oracle import mlp, step as ostep
    from oracle.inversion import GNOptions
    from workloads import Heat1D
    w = Heat1D(seed=args.seed)
    dec = crom.Decoder.from_layers(w.layers, w.m, precision="fp32", device=dev)
    st = crom.Stepper(dec, [0, w.n_samples], torch.from_numpy(w.samples).to(dev))
    opts = crom.GNOptions(max_iter=w.max_iter, tol_step=TOL_STEP["fp32"])
    q0 = np.asarray(w.ic, dtype=np.float64).copy()  # a generic starting latent (r = 3)
    q = [torch.from_numpy(q0[None].copy()).to(dev), torch.empty(1, w.r, dtype=torch.float64, device=dev)]
    nu = torch.tensor([w.nu], dtype=torch.float64, device=dev)
    for i in range(10):
        st.step(q[i % 2], nu, w.dt, opts, q_next=q[(i + 1) % 2])
    q[0].copy_(torch.from_numpy(q0[None].copy()))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.c1_steps):
        st.step(q[i % 2], nu, w.dt, opts, q_next=q[(i + 1) % 2])
    torch.cuda.synchronize()
    t_gpu = time.perf_counter() - t0
    q_gpu = q[args.c1_steps % 2].cpu().numpy()[0]
    out = {"workload": f"1D heat, nu {w.nu}, {w.n_samples} samples, dt {w.dt}, {args.c1_steps} GN steps "
                       f"(<= {w.max_iter} iterations), FP32",
           "gpu_s": t_gpu, "us_per_step": t_gpu / args.c1_steps * 1e6,
           "latent_steps_per_s": args.c1_steps / t_gpu}
    if args.c1_cpu:
        from threadpoolctl import threadpool_limits
        odec = mlp.MLPDecoder(w.layers, w.m)
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            qs, _ = ostep.heat_rollout(odec, w.samples.astype(np.float64), q0, w.nu, w.dt, args.c1_steps,
                                       GNOptions(max_iter=w.max_iter, tol_step=TOL_STEP["fp32"]))
            t_cpu = time.perf_counter() - t0
        out["oracle_cpu_s_1_thread"] = t_cpu
        out["gpu_vs_oracle_q_maxdiff"] = float(np.abs(q_gpu - qs[-1]).max())
        out["q_final_maxabs"] = float(np.abs(qs[-1]).max())
    return out


def config3_leg(args, crom, torch, dev):
    """3D neo-Hookean bar (decoder (3 + 16) -> 6 x ELU 256 -> 3, 500 samples
    of the 64 x 16 x 16 nodes, the face X_1 = 0 clamped, lam 1e4, mu 4e3,
    rho0 1000, gravity, dt 1e-3): one instance's latent step from a fixed
    state (Gauss-Newton with 5 iterations, and linearised), repeated, and the
    full-field decode of 16,384 nodes.  A point-eval is one sample through all 26 columns (value, 3
    gradient, 6 Hessian, 16 latent entries; 17,080,832 FLOP)."""
    from workloads import Elastic3D
    w = Elastic3D(seed=args.seed)
    X = w.nodes[w.sample_idx].astype(np.float32)
    clamp = (X[:, 0] == 0.0).astype(np.uint8)
    W3, D3, M3, R3 = 256, 6, 3, 16
    f_val = 2 * (M3 * W3 + (D3 - 1) * W3 * W3 + W3 * 3)
    f_tan = 2 * ((D3 - 1) * W3 * W3 + W3 * 3)
    f_pe = f_val + 25 * f_tan
    coef = torch.tensor([[w.lam, w.mu, w.rho0, *w.gravity]], dtype=torch.float64, device=dev)
    nodes = torch.from_numpy(w.nodes).to(dev)
    out = {"workload": f"neo-Hookean bar 64x16x16, {len(X)} samples, dt {w.dt}", "flop_per_point_eval": f_pe}
    for prec in (args.prec, "fp32") if args.prec != "fp32" else ("fp32",):
        dec = crom.Decoder.from_layers(w.layers, w.m, precision=prec, device=dev)
        st = crom.Stepper(dec, [0, len(X)], torch.from_numpy(X).to(dev), torch.from_numpy(clamp).to(dev),
                          pde="neohookean")
        res = {}
        for name, opts in (("gn", crom.GNOptions(max_iter=5, tol_step=TOL_STEP[prec])),
                           ("lls", crom.GNOptions(max_iter=1, linearized=True))):
            # every timed step starts from the same state (the untrained bar's
            # rollout would wander into degenerate latents within a few steps)
            q = torch.from_numpy(w.q0[None].copy()).to(dev)
            q_prev = q - 1e-3
            q_next = torch.empty_like(q)
            for _ in range(3):
                st.step(q, coef, w.dt, opts, q_next=q_next, q_prev=q_prev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.c3_steps):
                st.step(q, coef, w.dt, opts, q_next=q_next, q_prev=q_prev)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) / args.c3_steps
            inf = st.info()[0]
            fl = len(X) * (f_pe + (int(inf["ls_evals"]) + int(inf["iters"]) * R3) * f_tan) if not opts.linearized \
                else len(X) * f_pe
            res[name] = {"ms_per_step": t * 1e3, "latent_steps_per_s": 1.0 / t, "point_evals_per_s": fl / f_pe / t,
                         "achieved_tflops": fl / t / 1e12, "frac_of_peak": fl / t / 1e12 / PEAK[prec],
                         "gn_iters_last": int(inf["iters"]), "flags_last": int(inf["flags"])}
        g = torch.empty(len(nodes), 3, dtype=torch.float32, device=dev)
        qd = torch.from_numpy(w.q0).to(dev)
        for _ in range(3):
            dec.decode(nodes, qd, out=g)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            dec.decode(nodes, qd, out=g)
        e1.record()
        torch.cuda.synchronize()
        td = e0.elapsed_time(e1) * 1e-3 / 20
        res["full_field_decode"] = {"ms": td * 1e3, "achieved_tflops": len(nodes) * f_val / td / 1e12}
        out[prec] = res
    if args.c3_cpu:
        from oracle import elastic, mlp
        from oracle.inversion import GNOptions
        odec = mlp.MLPDecoder(w.layers, w.m)
        t0 = time.perf_counter()
        elastic.elastic_step(odec, X.astype(np.float64), w.q0, w.q0, w.lam, w.mu, w.rho0, w.gravity, w.dt,
                             GNOptions(max_iter=5, tol_step=TOL_STEP["fp32"]), clamp)
        out["oracle_cpu_s_per_gn_step"] = time.perf_counter() - t0
    return out


def guess_leg(args, crom, torch, dev, trained):
    """The encoder-based initial guess with the trained network and encoder:
    the 4 held-out diffusivities from the encoded initial field, 500 random
    interior samples of the 128 x 128 nodes, one step 20 times the rollout's
    (dt = 2e-3, a large change of the field), Gauss-Newton with at most 3
    iterations from q_n, and from the encoder's latent of the full-field
    update (crom_heat_guess over all 16,384 nodes, then crom_step_guess),
    with budgets of 1 and 3 iterations.  Reported per start: objective after
    the step, iterations, and the objective at the start; the guess's own
    cost is timed."""
    from workloads import rng as _rng
    w = trained["w"]
    nodes = trained["nodes"].to(torch.float32)
    P = nodes.shape[0]
    g = _rng(args.seed + 9)
    idx = np.arange(P).reshape(w.grid, w.grid)[1:-1, 1:-1].ravel()
    samples = nodes[torch.from_numpy(np.sort(g.choice(idx, size=500, replace=False))).to(dev)].contiguous()
    n = len(w.mu_test)
    dt = 20 * w.dt
    dec = crom.Decoder(trained["params"], w.m, w.r, w.d, w.width, w.depth, args.prec, dev)
    st = crom.Stepper(dec, np.arange(n + 1) * 500, samples.repeat(n, 1))
    nu = torch.from_numpy(np.asarray(w.mu_test, np.float64)).to(dev)
    q_n = torch.from_numpy(np.tile(trained["q0"], (n, 1))).to(dev)
    guess = crom.heat_guess(dec, trained["enc"], trained["hidden"], nodes, q_n, nu, dt)
    for _ in range(3):
        crom.heat_guess(dec, trained["enc"], trained["hidden"], nodes, q_n, nu, dt)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    e[0].record()
    for _ in range(10):
        crom.heat_guess(dec, trained["enc"], trained["hidden"], nodes, q_n, nu, dt)
    e[1].record()
    torch.cuda.synchronize()
    out = {"workload": f"{n} held-out diffusivities, 500 samples, one step of dt {dt}, Gauss-Newton <= 1 or 3 iterations",
           "guess_ms": e[0].elapsed_time(e[1]) / 10}
    for it in (1, 3):
        opts = crom.GNOptions(max_iter=it, tol_step=TOL_STEP[args.prec])
        for name, q_init in (("from_q_n", None), ("from_encoder_guess", guess)):
            st.step(q_n, nu, dt, opts, q_init=q_init)
            inf = st.info()
            out[f"{name}_{it}_iter"] = {"obj_last_mean": float(np.mean(inf["obj_last"])),
                                        "obj_first_mean": float(np.mean(inf["obj_first"])),
                                        "iters_mean": float(np.mean(inf["iters"])),
                                        "flags": [int(f) for f in inf["flags"]]}
    # the objective at the guess itself: a zero-iteration step from it
    st.step(guess, nu, dt, crom.GNOptions(max_iter=1, linearized=True))
    out["objective_at_guess_mean"] = float(np.mean(st.info()["obj_first"]))
    return out


def fe_leg(args, crom, torch, dev):
    """Corotated elasticity with finite-element forces: the falling bar of
    64 x 16 x 16 vertices as 85,050 jittered linear tetrahedra, 500 sample
    vertices and their one-ring, decoder (3 + 16) -> 6 x ELU 256 -> 3,
    mu ~ U(6e4, 7e4), lam = 0, rho0 1000, gravity, dt 1e-3: one instance's
    latent step from a fixed state (Gauss-Newton with 5 iterations, and
    linearised), repeated; the library's kernel timer gives the span from
    the set-up launch to the end of the inversion (ring decode, sample
    Jacobian, FE forces, inversion)."""
    from workloads import Corotated3D
    w = Corotated3D(seed=args.seed)
    sm = crom.FEStencil(w.X, w.tets, w.samples, dev)
    coef = torch.tensor([[w.lam, w.mu[0], w.rho0, *w.gravity]], dtype=torch.float64, device=dev)
    out = {"workload": f"corotated FE bar 64x16x16 ({w.tets.shape[0]} tetrahedra), {w.n_samples} samples, "
                       f"one-ring {sm.n_ring} vertices, {sm.n_inc} sample-tetrahedron pairs, dt {w.dt}"}
    for prec in (args.prec, "fp32") if args.prec != "fp32" else ("fp32",):
        dec = crom.Decoder.from_layers(w.layers, w.m, precision=prec, device=dev)
        st = crom.Stepper(dec, sm.offsets, sm.y, pde="corotated_fe", mesh=sm)
        res = {}
        for name, opts in (("gn", crom.GNOptions(max_iter=5, tol_step=TOL_STEP[prec])),
                           ("lls", crom.GNOptions(max_iter=1, linearized=True))):
            q = torch.from_numpy(w.q0.copy()).to(dev)
            q_prev = q - 1e-3
            q_next = torch.empty_like(q)
            for _ in range(3):
                st.step(q, coef, w.dt, opts, q_next=q_next, q_prev=q_prev)
            torch.cuda.synchronize()
            crom.kernel_timer(True)
            t0 = time.perf_counter()
            for _ in range(args.fe_steps):
                st.step(q, coef, w.dt, opts, q_next=q_next, q_prev=q_prev)
            torch.cuda.synchronize()
            t = (time.perf_counter() - t0) / args.fe_steps
            crom.kernel_timer(False)
            k_ms, k_n = crom.kernel_timer_read()
            inf = st.info()[0]
            res[name] = {"ms_per_step": t * 1e3, "latent_steps_per_s": 1.0 / t,
                         "kernels_ms_per_step": k_ms / max(1, k_n),
                         "gn_iters_last": int(inf["iters"]), "ls_evals_last": int(inf["ls_evals"]),
                         "flags_last": int(inf["flags"])}
        out[prec] = res
    return out


def single_leg(args, crom, torch, dev):
    """One instance of 2D heat (decoder (x in R^2, q in R^8) -> 5 ELU layers
    of width 128 -> 1, Xavier-uniform from a seed; mu ~ U(0.1, 1); 2,000
    samples uniform in (0, 1)^2; dt = 1e-4): per step the full-field decode
    of the 65,536 nodes of the 256 x 256 grid, then one latent step at the
    samples (Gauss-Newton, up to 5 iterations, the persistent step kernel);
    the steps form a rollout.  Latency-bound: one 16-sample batch per
    workgroup and dependent phases.  Reported in the headline's unit, with
    the step kernel's roofline, and the linearised step's rate."""
    from workloads import Heat2D
    wl = Heat2D(seed=args.seed)
    nodes = wl.nodes
    dec = crom.Decoder.from_layers(wl.layers, wl.m, precision=args.prec, device=dev)
    X = torch.from_numpy(nodes).to(dev)
    st = crom.Stepper(dec, [0, wl.n_samples], torch.from_numpy(wl.samples).to(dev))
    q = [torch.from_numpy(wl.q0[None].copy()).to(dev), torch.empty(1, R, dtype=torch.float64, device=dev)]
    nu = torch.tensor([wl.mu], dtype=torch.float64, device=dev)
    g = torch.empty(len(nodes), 1, dtype=torch.float32, device=dev)
    opts = crom.GNOptions(max_iter=5, tol_step=TOL_STEP[args.prec])

    # The decode and the step run one after the other on one stream (a
    # second stream for the decode slowed the persistent step kernel: its
    # per-phase latency suffers from co-running workgroups).
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
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    crom.kernel_timer(True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        one(args.warmup + i, evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    crom.kernel_timer(False)
    k_ms, k_n = crom.kernel_timer_read()
    t_dec = np.array([e[0].elapsed_time(e[1]) for e in evs]) * 1e-3
    t_step = np.array([e[1].elapsed_time(e[2]) for e in evs]) * 1e-3
    # the same rollout again, untimed, reading every step's outcome
    q[0].copy_(torch.from_numpy(wl.q0[None].copy()))
    for i in range(args.warmup):
        one(i)
    flop_step, its, lse, flags = 0.0, [], [], 0
    for i in range(args.steps):
        one(args.warmup + i)
        inf = st.info()[0]
        its.append(int(inf["iters"]))
        lse.append(int(inf["ls_evals"]))
        flags |= int(inf["flags"])
        flop_step += step_flops(wl.n_samples, int(inf["iters"]), int(inf["ls_evals"]))
    torch.cuda.synchronize()
    flop_dec = args.steps * len(nodes) * FLOP_VALUE_COL
    t_kernel = k_ms * 1e-3 / max(1, k_n)
    fl = flop_step / args.steps
    achieved = fl / t_kernel / 1e12
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
    return {"workload": "2D heat, 256x256 grid: full-field decode of 65,536 nodes + one Gauss-Newton latent "
                        "step at 2,000 samples per step, one instance, Xavier-uniform network",
            "precision": args.prec, "gn_tol_step": TOL_STEP[args.prec],
            "point_evals_per_s": (flop_dec + flop_step) / FLOP_POINT_EVAL_LLS / wall,
            "ms_per_step": wall / args.steps * 1e3, "latent_steps_per_s": args.steps / wall,
            "lls_latent_steps_per_s": args.steps / (time.perf_counter() - t1),
            "step_ms_avg": t_step.mean() * 1e3, "decode_ms_avg": t_dec.mean() * 1e3,
            "gn_iters_mean": float(np.mean(its)), "ls_evals_mean": float(np.mean(lse)), "flags_or": flags,
            "step_kernel": {"avg_ms": t_kernel * 1e3, "flop_per_launch": fl, "achieved_tflops": achieved,
                            "frac": achieved / PEAK[args.prec],
                            "traffic": measured_traffic("step_kernel")},
            "decode_kernel": {"avg_ms": t_dec.mean() * 1e3,
                              "achieved_tflops": len(nodes) * FLOP_VALUE_COL / t_dec.mean() / 1e12}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--prec", default="bf16", choices=sorted(PEAK))
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="host seconds for the oracle's sample of the headline workload (0: skip)")
    ap.add_argument("--single", type=int, default=1, help="the single-instance 2D heat leg (0: skip)")
    ap.add_argument("--modes", default="", help="comma list of batched modes to run (e.g. bf16_lls; default all four)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--train-time-steps", type=int, default=50)
    ap.add_argument("--train-precs", default="bf16,fp32", help="arithmetic of the timed training steps")
    ap.add_argument("--train-conv", type=int, default=1, help="time the convolutional-encoder training step")
    ap.add_argument("--train-steps", type=int, default=20000,
                    help="BF16 training run whose network the batched leg rolls out (0: untrained)")
    ap.add_argument("--judge", type=int, default=8, help="instances whose rollout error the FD solver judges")
    ap.add_argument("--c1-steps", type=int, default=1000, help="1D heat rollout length (0: skip)")
    ap.add_argument("--c1-cpu", type=int, default=1, help="time the oracle's 1D rollout too")
    ap.add_argument("--c3-steps", type=int, default=20, help="3D elastic steps timed (0: skip)")
    ap.add_argument("--c3-cpu", type=int, default=0, help="time one oracle elastic step too (about 30 s)")
    ap.add_argument("--fe-steps", type=int, default=20, help="corotated FE steps timed (0: skip)")
    ap.add_argument("--siren", type=int, default=1, help="time the sine-activated decoder and step (0: skip)")
    ap.add_argument("--sampling-rounds", type=int, default=32,
                    help="greedy sample-selection rounds with the trained network (0: skip)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="copy this many MiB once, untimed (a known-size kernel for counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("this benchmark runs on one GPU: the instances of a batch are independent and the "
              "step of one instance is not split across devices", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2206_02607_amd import crom

    dev = torch.device("cuda:0")
    if args.copy_probe_mib > 0:  # a copy of known size for the counter calibration
        src = torch.empty(args.copy_probe_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    training, trained = train_leg(args, crom, torch, dev) if args.train_time_steps > 0 else (None, None)
    batched = batched_leg(args, crom, torch, dev, trained)
    single = single_leg(args, crom, torch, dev) if args.single else None
    c1 = config1_leg(args, crom, torch, dev) if args.c1_steps > 0 else None
    c3 = config3_leg(args, crom, torch, dev) if args.c3_steps > 0 else None
    sampling = sampling_leg(args, crom, torch, dev, trained) if trained and args.sampling_rounds > 0 else None
    guess = guess_leg(args, crom, torch, dev, trained) if trained else None
    siren = siren_leg(args, crom, torch, dev) if args.siren else None
    fe = fe_leg(args, crom, torch, dev) if args.fe_steps > 0 else None

    head = batched["modes"][batched["headline_mode"]]
    prec, lin = head["precision"], head["inversion"] == "linearised"
    kernel_s = head["timed_kernels_ms"] * 1e-3
    achieved = head["flop_per_step"] / kernel_s / 1e12
    roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK[prec], "unit": "TFLOP/s",
            "frac": achieved / PEAK[prec],
            "traffic": measured_traffic("lls_jets_kernel", "traffic_batched_2d_heat.json") if lin else None,
            "kernel": head["timed_kernels"], "avg_ms": head["timed_kernels_ms"],
            "flop_per_launch": head["flop_per_step"],
            "flop_unit": ("658,944 algorithmic FLOP per point-eval (the 2D decoder: value, 2 x tangents and "
                          "Laplacian forward, the latent Jacobian by one adjoint column and the first layer's "
                          "latent columns; folded first layer, no padding) x the point-evals of one step" if lin
                          else "658,944 FLOP per sample for the evaluation at q_n, 133,120 per further adjoint "
                               "column (iteration) and 131,328 per difference column (trial), over the step")}
    cpu = None
    if args.cpu_seconds > 0:
        from workloads import Batched2D
        kw = {"max_iter": 1, "linearized": True} if lin else {"max_iter": 5, "tol_step": TOL_STEP["fp32"]}
        cpu = cpu_baseline_batched(Batched2D(seed=args.seed), kw, args.cpu_seconds)
    out = {
        "metric": "decoder+Jacobian point-evals/sec and latent steps/sec at fixed rollout error",
        "value": head["point_evals_per_s"], "unit": "point-evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"bf16": "bf16", "fp32": "fp32", "bf16x3": "bf16", "bf16pure": "bf16"}[prec],
        "data": "synthetic",
        "config": {"workload": "batched rollout of 512 2D heat instances (mu_i ~ U(0.1, 1), S_i ~ U{200..2000} "
                               "samples of the 128x128 lattice, r = 8, dt = 1e-4), trained network, one latent "
                               "step of every instance per step",
                   "mode": batched["headline_mode"], "mode_rule": batched["headline_rule"],
                   "precision": prec, "inversion": head["inversion"]},
        "latent_steps_per_s": head["instance_steps_per_s"],
        "rollout_error": head.get("rollout_error_mean"),
        "roofline": roof,
        "cpu_baseline": cpu,
        "batched": batched,
        "heat2d_single": single,
        "heat1d": c1,
        "elastic3d": c3,
        "training": training,
        "sampling": sampling,
        "encoder_guess": guess,
        "siren": siren,
        "corotated_fe": fe,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
