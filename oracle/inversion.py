"""Network inversion in FP64 (test infrastructure only).

The latent vector at the next step minimises the squared mismatch between
the decoder at the samples and the updated field (eq. "invert", Sec. "Step 3:
Network Inversion"; Sec. "Network Inversion").  The paper solves it with
Gauss-Newton plus a standard backtracking line search, starting from the
previous latent vector (Sec. "Initial Guess for the Nonlinear Solver"), or
with one linearised solve of the normal equations (Sec. "Linearization").

Readings where the paper gives no constants (all taken from the textbook
backtracking scheme, Nocedal & Wright, Alg. 3.1):
* objective phi(q) = 1/2 * ||f - g(q)||^2 over all samples and outputs;
* search direction: the normal-equation solution (J^T J) delta = J^T rho with
  rho = f - g(q_i), solved by Cholesky;
* trial steps alpha = 1, shrink, shrink^2, ... with at most ``ls_max``
  shrinks; accept the first alpha with
  phi(q_i + alpha delta) <= phi(q_i) - c * alpha * (J^T rho) . delta;
* stop without moving when the Gauss-Newton step itself is negligible,
  ||delta|| <= tol * (1 + ||q_i||) (no line search is tried then: at that
  size no decrease of phi can be resolved in floating point);
* stop after an accepted step with alpha * ||delta|| <= tol * (1 + ||q_i||),
  or after ``max_iter`` accepted steps (flag MAXITER);
* Cholesky declares the system singular when a pivot (the value under the
  square root) is not above 1e-14 * max(diag A); the iterate is then kept;
* the linearised variant is one Gauss-Newton step with alpha = 1 forced.

Status flags (bit values shared with the C interface by definition, not by
code): MAXITER 1, SINGULAR 2, NONFINITE 4, LS_FAIL 8, INVERTED 32 (16 is the
GPU's ABORTED, which has no counterpart here).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

MAXITER, SINGULAR, NONFINITE, LS_FAIL, INVERTED = 1, 2, 4, 8, 32
PIVOT_REL = 1e-14


@dataclass
class GNOptions:
    max_iter: int = 5
    linearized: bool = False
    ls_max: int = 10
    tol_step: float = 1e-10
    armijo_c: float = 1e-4
    ls_shrink: float = 0.5


@dataclass
class GNInfo:
    flags: int = 0
    iters: int = 0
    ls_evals: int = 0
    obj_first: float = float("nan")
    obj_last: float = float("nan")


def cholesky(A: np.ndarray, pivot_rel: float = PIVOT_REL):
    """Lower-triangular L with L L^T = A, or None when a pivot is not above
    pivot_rel * max(diag A) (or is not finite)."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    dmax = float(np.max(np.diag(A))) if n else 0.0
    thresh = pivot_rel * dmax
    L = np.zeros_like(A)
    for j in range(n):
        s = A[j, j] - np.dot(L[j, :j], L[j, :j])
        if not np.isfinite(s) or s <= thresh:
            return None
        L[j, j] = np.sqrt(s)
        for i in range(j + 1, n):
            L[i, j] = (A[i, j] - np.dot(L[i, :j], L[j, :j])) / L[j, j]
    return L


def chol_solve(L: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Solve L L^T x = b by forward then backward substitution."""
    n = L.shape[0]
    y = np.zeros(n)
    for i in range(n):
        y[i] = (b[i] - np.dot(L[i, :i], y[:i])) / L[i, i]
    x = np.zeros(n)
    for i in reversed(range(n)):
        x[i] = (y[i] - np.dot(L[i + 1:, i], x[i + 1:])) / L[i, i]
    return x


def normal_equations(J: np.ndarray, rho: np.ndarray):
    """A = J^T J, b = J^T rho, phi = 1/2 rho^T rho for stacked J [N, r]."""
    return J.T @ J, J.T @ rho, 0.5 * float(rho @ rho)


def gauss_newton(value_fn, value_jac_fn, target: np.ndarray, q0: np.ndarray,
                 opts: GNOptions):
    """Minimise 1/2 ||target - value(q)||^2 from q0.

    value_fn(q) -> stacked decoder values [N]; value_jac_fn(q) -> (values [N],
    Jacobian [N, r]).  Returns (q, GNInfo)."""
    q = np.asarray(q0, dtype=np.float64).copy()
    target = np.asarray(target, dtype=np.float64).ravel()
    info = GNInfo()
    g, J = value_jac_fn(q)
    rho = target - g
    A, b, phi = normal_equations(J, rho)
    info.obj_first = phi
    info.obj_last = phi
    for it in range(opts.max_iter):
        if not (np.isfinite(phi) and np.all(np.isfinite(A)) and np.all(np.isfinite(b))):
            info.flags |= NONFINITE
            break
        L = cholesky(A)
        if L is None:
            info.flags |= SINGULAR
            break
        delta = chol_solve(L, b)
        if opts.linearized:
            q = q + delta
            info.iters = 1
            break
        if float(np.linalg.norm(delta)) <= opts.tol_step * (1.0 + float(np.linalg.norm(q))):
            break
        slope = float(b @ delta)
        alpha = 1.0
        accepted = False
        for _ in range(opts.ls_max + 1):
            qt = q + alpha * delta
            gt = value_fn(qt)
            info.ls_evals += 1
            rt = target - gt
            phit = 0.5 * float(rt @ rt)
            if np.isfinite(phit) and phit <= phi - opts.armijo_c * alpha * slope:
                accepted = True
                break
            alpha *= opts.ls_shrink
        if not accepted:
            info.flags |= LS_FAIL
            break
        step = alpha * float(np.linalg.norm(delta))
        qnorm = float(np.linalg.norm(q))
        q = qt
        info.iters += 1
        g, J = value_jac_fn(q)
        rho = target - g
        A, b, phi = normal_equations(J, rho)
        info.obj_last = phi
        if step <= opts.tol_step * (1.0 + qnorm):
            break
    else:
        info.flags |= MAXITER
    return q, info


def gauss_newton_from_guess(value_fn, value_jac_fn, target: np.ndarray, q_n: np.ndarray, q_guess,
                            opts: GNOptions):
    """Gauss-Newton with a second candidate starting point (Sec. "Initial
    Guess for the Nonlinear Solver": the previous latent is the natural start;
    where the field changes a lot over a step, an encoder's latent for the
    updated field can be the better one).

    Readings (the paper gives no rule for combining the two):
    * the guess is considered only when q_n is not already a stationary
      point: the normal equations at q_n are finite and solvable and their
      step is not negligible (the stopping test of ``gauss_newton``);
    * the guess replaces q_n as the start when its objective is finite and
      strictly smaller than q_n's; otherwise Gauss-Newton runs from q_n as
      without a guess;
    * the linearised variant (one step from q_n) ignores the guess;
    * obj_first stays the objective at q_n.
    Returns (q, GNInfo, used_guess)."""
    if q_guess is None or opts.linearized:
        q, info = gauss_newton(value_fn, value_jac_fn, target, q_n, opts)
        return q, info, False
    target = np.asarray(target, dtype=np.float64).ravel()
    q_n = np.asarray(q_n, dtype=np.float64)
    g, J = value_jac_fn(q_n)
    A, b, phi = normal_equations(J, target - g)
    usable = np.isfinite(phi) and np.all(np.isfinite(A)) and np.all(np.isfinite(b))
    L = cholesky(A) if usable else None
    if L is not None:
        delta = chol_solve(L, b)
        if float(np.linalg.norm(delta)) > opts.tol_step * (1.0 + float(np.linalg.norm(q_n))):
            rg = target - value_fn(np.asarray(q_guess, dtype=np.float64))
            phig = 0.5 * float(rg @ rg)
            if np.isfinite(phig) and phig < phi:
                q, info = gauss_newton(value_fn, value_jac_fn, target, q_guess, opts)
                info.obj_first = phi
                return q, info, True
    q, info = gauss_newton(value_fn, value_jac_fn, target, q_n, opts)
    return q, info, False
