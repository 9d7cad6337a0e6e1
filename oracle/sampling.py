"""Robust greedy selection of the integration samples in FP64 (test
infrastructure only).

Appendix "Robust Sampling", Alg. "Robust sampling".  The integration samples
are a subset M of the nodes x_1 .. x_P of the full-order discretisation.
One round of the greedy loop:

1. the residual vector of M (the algorithm's Calculate_Residual): for every
   training parameter mu_k, the latent dynamics run with the samples M from
   the initial latent to the final time; the final latent q_end(mu_k) is
   decoded at every node, and
       res[i] = sum_k | g(x_i, q_end(mu_k)) - f(x_i, t_end; mu_k) |
   with f the full-order solution;
2. if Metric(res) = mean(res) + max(res) is below the target, M is the
   result;
3. otherwise the n_try nodes with the largest individual residuals are the
   candidates; each candidate c gives the residual vector of M + {c}, and the
   candidate whose vector has the smallest metric joins M.

Readings where the algorithm is silent:
* candidates are nodes outside M (adding a member leaves M as it is);
* the largest residuals are ranked by value, ties to the lower node index;
  the smallest metric is taken by value, ties to the earlier candidate in
  that ranking; NaN ranks above every number in both;
* |.| is the Euclidean norm over the d output components;
* the residual vector of M + {c} for the chosen c is the residual vector of
  the next round's set (the same computation, so it is not repeated);
* the loop also ends when M holds max_samples nodes or no node is left to
  try, and reports whether the target was met.

Parity status: pinned by ``tests/test_oracle_sampling.py`` (a decoder linear
in q, whose linearised rollout is a matrix power of a pseudo-inverse, gives
the residual in closed form; brute force over every candidate fixes the
greedy choice).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Sequence

import numpy as np

from .step import heat_rollout


def metric(res: np.ndarray) -> float:
    """Metric(res) = mean(res) + max(res)."""
    r = np.asarray(res, dtype=np.float64)
    return float(r.mean() + r.max())


def _rank_key(v: float) -> float:
    return np.inf if np.isnan(v) else float(v)


def max_indices(res: np.ndarray, members: Sequence[int], n: int) -> List[int]:
    """The n nodes outside `members` with the largest residuals (ties to the
    lower index, NaN first)."""
    excluded = set(int(i) for i in members)
    order = sorted((i for i in range(len(res)) if i not in excluded),
                   key=lambda i: (-_rank_key(res[i]), i))
    return order[:n]


def min_index(values: Sequence[float]) -> int:
    """Position of the smallest value (the first one on ties; NaN last)."""
    best = 0
    for i in range(1, len(values)):
        if _rank_key(values[i]) < _rank_key(values[best]):
            best = i
    return best


def residual(decoder, nodes: np.ndarray, ref: np.ndarray, samples: Sequence[int],
             final_latent: Callable[[int, Sequence[int]], np.ndarray]) -> np.ndarray:
    """Residual vector res [P] of the sample set `samples` (node indices).

    nodes [P, m]; ref [n_mu, P, d] (or [n_mu, P] for d = 1) the full-order
    field at the final time per training parameter; final_latent(k, samples)
    -> the final latent of parameter k's rollout with those samples."""
    P = nodes.shape[0]
    ref = np.asarray(ref, dtype=np.float64).reshape(ref.shape[0], P, -1)
    res = np.zeros(P)
    for k in range(ref.shape[0]):
        q = final_latent(k, list(samples))
        g = np.asarray(decoder.value(nodes, q), dtype=np.float64).reshape(P, -1)
        res += np.sqrt(((g - ref[k]) ** 2).sum(axis=1))
    return res


def heat_final_latent(decoder, nodes: np.ndarray, q0: np.ndarray, nus: Sequence[float], dt: float,
                      n_steps: int, opts, clamp=None) -> Callable[[int, Sequence[int]], np.ndarray]:
    """final_latent for the heat equation: n_steps latent steps of parameter
    k (diffusivity nus[k], initial latent q0[k]) with the samples given by
    node index; clamp [P] marks Dirichlet nodes (or None)."""
    q0 = np.asarray(q0, dtype=np.float64).reshape(len(nus), -1)

    def run(k: int, samples: Sequence[int]) -> np.ndarray:
        idx = np.asarray(samples, dtype=np.int64)
        c = None if clamp is None else np.asarray(clamp)[idx]
        traj, _ = heat_rollout(decoder, nodes[idx], q0[k], float(nus[k]), dt, n_steps, opts, c)
        return traj[-1]

    return run


@dataclass
class SamplingResult:
    samples: List[int]          # M in the order the nodes joined it
    metric: float               # Metric of the residual vector of the returned M
    reached: bool               # metric < target
    residual: np.ndarray        # residual vector of the returned M
    candidates: List[List[int]] = field(default_factory=list)   # per round
    metrics: List[List[float]] = field(default_factory=list)    # per round, per candidate


def robust_sampling(decoder, nodes: np.ndarray, ref: np.ndarray, init: Sequence[int],
                    final_latent: Callable[[int, Sequence[int]], np.ndarray], target: float,
                    n_try: int = 10, max_samples: int = 10 ** 9) -> SamplingResult:
    """The greedy loop of Alg. "Robust sampling" from the initial set `init`."""
    M = [int(i) for i in init]
    res = residual(decoder, nodes, ref, M, final_latent)
    out = SamplingResult(M, metric(res), False, res)
    while True:
        m = metric(res)
        out.metric, out.residual = m, res
        if m < target:
            out.reached = True
            break
        if len(M) >= max_samples:
            break
        cand = max_indices(res, M, n_try)
        if not cand:
            break
        results = [residual(decoder, nodes, ref, M + [c], final_latent) for c in cand]
        metrics = [metric(r) for r in results]
        j = min_index(metrics)
        out.candidates.append(cand)
        out.metrics.append(metrics)
        M.append(cand[j])
        res = results[j]
    out.samples = M
    return out
