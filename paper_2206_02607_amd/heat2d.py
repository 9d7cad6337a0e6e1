"""2D heat end to end on the GPU: full-order FP64 snapshots, decoder
training, latent rollout and its error against the full-order solution.

Every computation runs in the library (crom_fd_heat, crom_train_step,
crom_encode, crom_step, crom_decode); this module only sequences the calls
(Sec. "Manifold Construction" for the training data and loss, Sec. "Method:
Latent Space Dynamics" for the rollout, the image-diffusion experiment's
full-order model for the snapshots)."""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import crom


def fd_snapshots(u0: np.ndarray, mus: Sequence[float], times: Sequence[float], dx: float, dt_fd: float,
                 device="cuda") -> torch.Tensor:
    """FP64 fields [n_mu, n_times, nx, ny] of u_t = mu Lap u from the shared
    initial field u0 [nx, ny], recorded at `times` (multiples of dt_fd)."""
    n_mu = len(mus)
    u = torch.from_numpy(np.ascontiguousarray(u0, dtype=np.float64)).to(device)
    u = u.unsqueeze(0).repeat(n_mu, 1, 1).contiguous()
    nu = torch.as_tensor(np.asarray(mus, dtype=np.float64), device=device)
    scratch = torch.empty_like(u)
    out = torch.empty(n_mu, len(times), *u0.shape, dtype=torch.float64, device=device)
    t_prev = 0
    for k, t in enumerate(times):
        steps = int(round(t / dt_fd))
        if steps < t_prev:
            raise ValueError("times must be non-decreasing")
        crom.fd_heat(u, nu, dx, dt_fd, steps - t_prev, scratch)
        out[:, k] = u
        t_prev = steps
    return out


# Learning-rate schedule of Sec. "Training Details": 10, 5, 2, 1, 0.5 and
# 0.2 times a base rate, in equal stages (the base rate 1e-4 makes the
# first stage 1e-3).
LR_STAGES = (10.0, 5.0, 2.0, 1.0, 0.5, 0.2)


def lr_at(step: int, steps: int, base: float = 1e-4) -> float:
    return base * LR_STAGES[min(len(LR_STAGES) - 1, step * len(LR_STAGES) // max(1, steps))]


class Standardization:
    """The standardization of the training data (Sec. "Training Details"):
    u_s = (u - u_mean) / u_std over the whole training set, x_s =
    (x - x_mean) / x_std per coordinate over the nodes (population moments).
    The moments live on the device (crom_standardization); the library
    computes them, applies them and folds them into the trained networks."""

    def __init__(self, s: torch.Tensor, m: int):
        self.s = s
        self.m = m

    @classmethod
    def of(cls, snaps: torch.Tensor, nodes: torch.Tensor) -> "Standardization":
        return cls(crom.standardization_of(snaps, nodes), nodes.shape[1])

    def values(self) -> dict:
        """The moments on the host (synchronises; for reports)."""
        v = self.s.cpu().numpy()
        return {"u_mean": float(v[0]), "u_std": float(v[1]), "x_mean": v[2:2 + self.m].copy(),
                "x_std": v[5:5 + self.m].copy()}

    def data(self, snaps: torch.Tensor) -> torch.Tensor:
        return crom.standardize(self.s, u=snaps)[0]

    def points(self, nodes: torch.Tensor) -> torch.Tensor:
        return crom.standardize(self.s, x=nodes)[1]

    def fold(self, dec: crom.Decoder, enc_params: torch.Tensor, n_in: int, hidden: int,
             enc_kind: str = "dense") -> None:
        """Rewrite the trained decoder and encoder in place so that they act
        on physical points and fields: g(x, q) = u_std g_s(x_s, q) + u_mean
        and e(u) = e_s(u_s) (crom_fold_standardization; re-packs the decoder)."""
        crom.fold_standardization(dec, self.s, enc_params, n_in, hidden, enc_kind)


def train(trainer: crom.Trainer, snaps: torch.Tensor, steps: int, base_lr: float = 1e-4, seed: int = 0,
          log_every: int = 0) -> np.ndarray:
    """Adam steps over shuffled batches of the snapshot rows snaps [N, P]
    (FP32 on the device; each epoch is a seeded permutation, a short last
    batch rolls into the next epoch), with the staged learning rate.
    Returns the batch losses."""
    gen = np.random.Generator(np.random.PCG64(seed))
    N, B = snaps.shape[0], trainer.B
    order = np.empty(0, dtype=np.int64)
    losses = torch.empty(steps, dtype=torch.float32, device=snaps.device)
    for s in range(steps):
        if order.size < B:
            order = np.concatenate([order, gen.permutation(N)])
        idx, order = order[:B], order[B:]
        batch = snaps[torch.from_numpy(idx).to(snaps.device)]
        losses[s] = trainer.step(batch, lr_at(s, steps, base_lr))[0]
        if log_every and (s + 1) % log_every == 0:
            print(f"  train step {s + 1}: loss {losses[s].item():.3e}", flush=True)
    return losses.cpu().numpy()


@dataclass
class Rollout:
    steps: List[int]
    q: List[np.ndarray]        # [n_inst, r] at each recorded step
    flags: List[np.ndarray]    # OR of the flags of every step up to each recorded step
    iters: float               # mean Gauss-Newton iterations per instance-step
    fallbacks: np.ndarray = None  # steps per instance taken by the full-order fallback


def rollout(dec: crom.Decoder, q0: np.ndarray, y: np.ndarray, mus: Sequence[float], dt: float, n_steps: int,
            opts: crom.GNOptions, record: Sequence[int], offsets: Optional[np.ndarray] = None,
            fallback: Optional[crom.HeatFallback] = None) -> Rollout:
    """Latent steps for len(mus) instances from q0 [n_inst, r]; records q
    after the steps listed in `record`.  Samples: y [S, m] shared by every
    instance, or with `offsets` [n_inst + 1] the CSR rows of y per instance.
    With `fallback`, an instance whose step failed (SINGULAR, NONFINITE,
    LS_FAIL) takes the full-order fallback's latent for that step instead
    (decode at every node, finite-difference update over dt, projection
    back onto the decoder); Rollout.fallbacks counts them per instance."""
    n = len(mus)
    if offsets is None:
        S = y.shape[0]
        offsets = np.arange(n + 1, dtype=np.int64) * S
        y = np.tile(np.asarray(y, np.float32), (n, 1))
    yy = torch.from_numpy(np.asarray(y, np.float32)).to(dec.params.device)
    st = crom.Stepper(dec, np.asarray(offsets, np.int64), yy)
    q = torch.from_numpy(np.asarray(q0, np.float64).reshape(n, dec.r)).to(dec.params.device)
    q_next = torch.empty_like(q)
    flags = np.zeros(n, dtype=np.int32)
    out = Rollout([], [], [], 0.0, np.zeros(n, dtype=np.int64))
    nu_dev = torch.as_tensor(np.asarray(mus, np.float64), device=dec.params.device)
    rec = set(record)
    iters = 0
    if 0 in rec:
        out.steps.append(0)
        out.q.append(q.cpu().numpy())
        out.flags.append(flags.copy())
    for k in range(1, n_steps + 1):
        st.step(q, mus, dt, opts, q_next)
        q, q_next = q_next, q
        inf = st.info()  # every step's outcome (one synchronisation per step)
        flags |= inf["flags"]
        iters += int(inf["iters"].sum())
        if fallback is not None:
            failed = np.flatnonzero(inf["flags"] & crom.FLAGS_FAILED)
            if failed.size:
                fallback(failed, q_next, nu_dev, dt, q)  # q_next holds this step's q_n after the swap
                out.fallbacks[failed] += 1
        if k in rec:
            out.steps.append(k)
            out.q.append(q.cpu().numpy())
            out.flags.append(flags.copy())
    out.iters = iters / max(1, n_steps) / n
    return out


def decode_fields(dec: crom.Decoder, nodes: torch.Tensor, q: np.ndarray) -> torch.Tensor:
    """Decoded fields [n_inst, P] at the nodes for latents q [n_inst, r]."""
    out = torch.empty(q.shape[0], nodes.shape[0], dtype=torch.float32, device=nodes.device)
    for i in range(q.shape[0]):
        dec.decode(nodes, torch.from_numpy(np.asarray(q[i], np.float64)), out=out[i].view(-1, 1))
    return out


def rel_error(approx: torch.Tensor, ref: torch.Tensor) -> np.ndarray:
    """Relative L2 error per row: |approx - ref| / |ref|."""
    a = approx.to(torch.float64)
    r = ref.to(torch.float64).reshape(a.shape)
    return ((a - r).norm(dim=1) / r.norm(dim=1)).cpu().numpy()


def spacetime_error(approx: Sequence[torch.Tensor], ref: Sequence[torch.Tensor]) -> np.ndarray:
    """Relative L2 error over a trajectory, per instance:
    sqrt(sum_t |a_t - r_t|^2) / sqrt(sum_t |r_t|^2), for lists of [n_inst, P]."""
    num = sum(((a.to(torch.float64) - r.to(torch.float64).reshape(a.shape)) ** 2).sum(dim=1)
              for a, r in zip(approx, ref))
    den = sum((r.to(torch.float64).reshape(a.shape) ** 2).sum(dim=1) for a, r in zip(approx, ref))
    return (num.sqrt() / den.sqrt()).cpu().numpy()
