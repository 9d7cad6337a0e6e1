"""Neo-Hookean elastodynamics at the integration samples in FP64 (test
infrastructure only).

Sec. "Solid Mechanics / Continuous PDE": rho0 phi_tt = div P(grad phi) +
rho0 B, with the deformation map phi = X + u.  The reduced model represents
the displacement u(X, t) = g(X, q(t)) (Sec. "Solid Mechanics / Reduced-order
Model") and takes the velocity from the tangent space of the manifold,
phi_t = (dg/dq) qdot with qdot_n = (q_n - q_{n-1}) / dt and qdot_0 = 0.

Readings (the paper's own solids use corotated elasticity with forces from a
tetrahedral mesh; the workload fixes a neo-Hookean bar and network
derivatives):
* compressible neo-Hookean first Piola-Kirchhoff stress
  P = mu (F - F^-T) + lam ln(J) F^-T, the derivative of the energy density
  Psi = mu/2 (tr F^T F - 3) - mu ln J + lam/2 (ln J)^2;
* F = I + du/dX from the network's x-gradient, and the divergence through
  the network's x-Hessian: (div P)_i = sum_{j,k,l} dP_ij/dF_kl d2u_k/dX_l dX_j;
* symplectic Euler at the samples: v+ = v + dt (div P / rho0 + B),
  u+ = u + dt v+; a clamped sample targets u+ = 0;
* the inversion then projects u+ onto the decoder exactly as for heat;
* det F <= 0 at a sample whose update uses the stress (not clamped) has no
  neo-Hookean energy (ln J): the step reports INVERTED, and its NaN targets
  make the inversion stop with NONFINITE at q_n.
"""
from __future__ import annotations

import numpy as np

from .inversion import INVERTED, GNOptions
from .step import invert


def energy(F: np.ndarray, lam: float, mu: float) -> float:
    """Neo-Hookean energy density of one deformation gradient F [3, 3]."""
    J = np.linalg.det(F)
    lnJ = np.log(J)
    return 0.5 * mu * (np.sum(F * F) - 3.0) - mu * lnJ + 0.5 * lam * lnJ ** 2


def _inv(F: np.ndarray) -> np.ndarray:
    """F^-1 for F [.., 3, 3]; NaN where F is exactly singular (det F = 0 is
    an inverted sample: no stress, NaN like ln J of det F < 0)."""
    F = np.asarray(F, dtype=np.float64)
    flat = F.reshape(-1, 3, 3)
    out = np.full_like(flat, np.nan)
    ok = np.linalg.det(flat) != 0.0
    out[ok] = np.linalg.inv(flat[ok])
    return out.reshape(F.shape)


def _ln_det(F: np.ndarray) -> np.ndarray:
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.log(np.linalg.det(F))


def pk1(F: np.ndarray, lam: float, mu: float) -> np.ndarray:
    """First Piola-Kirchhoff stress P(F) [.., 3, 3] for F [.., 3, 3]."""
    FinvT = np.swapaxes(_inv(F), -1, -2)
    lnJ = _ln_det(F)[..., None, None]
    return mu * (F - FinvT) + lam * lnJ * FinvT


def dpk1(F: np.ndarray, lam: float, mu: float) -> np.ndarray:
    """dP_ij / dF_kl [.., 3, 3, 3, 3] (written out from P's three terms:
    d F = I (x) I, d F^-T_ij / d F_kl = -Finv_jk Finv_li, d ln J / d F_kl =
    Finv_lk)."""
    Fi = _inv(F)
    lnJ = _ln_det(F)[..., None, None, None, None]
    eye = np.eye(3)
    t1 = np.einsum("ik,jl->ijkl", eye, eye)
    t2 = np.einsum("...jk,...li->...ijkl", Fi, Fi)
    t3 = np.einsum("...lk,...ji->...ijkl", Fi, Fi)
    return mu * t1 + (mu - lam * lnJ) * t2 + lam * t3


def div_pk1(F: np.ndarray, hess: np.ndarray, lam: float, mu: float) -> np.ndarray:
    """(div P)_i = sum_{j,k,l} dP_ij/dF_kl d2u_k/(dX_l dX_j); F [S, 3, 3],
    hess [S, 3, 3, 3] with hess[s, k, l, j] = d2u_k / dX_l dX_j."""
    return np.einsum("sijkl,sklj->si", dpk1(F, lam, mu), hess)


def elastic_targets(decoder, X: np.ndarray, q_n: np.ndarray, q_prev, lam: float, mu: float,
                    rho0: float, B, dt: float, clamp=None):
    """Targets u+ [S, 3] at the samples X [S, 3] and the increments
    rho0 = u+ - u(q_n) [S, 3] (formed directly, dt v+, or -u when clamped).
    decoder.jets(X, q) -> (u [S,3], du/dX [S,3,3], d2u/dX2 [S,3,3,3],
    du/dq [S,3,r]); q_prev None means qdot = 0."""
    u, G, H, Jq = decoder.jets(X, q_n)
    F = np.eye(3)[None] + G
    qdot = np.zeros_like(q_n) if q_prev is None else (np.asarray(q_n) - np.asarray(q_prev)) / dt
    v = np.einsum("skr,r->sk", Jq, qdot)
    acc = div_pk1(F, H, lam, mu) / rho0 + np.asarray(B, dtype=np.float64)[None, :]
    v_next = v + dt * acc
    inc = dt * v_next
    if clamp is not None:
        c = np.asarray(clamp, dtype=bool)
        inc = np.where(c[:, None], -u, inc)
    return u + inc, inc


def inverted(decoder, X: np.ndarray, q_n: np.ndarray, clamp=None) -> bool:
    """Whether det(I + du/dX) <= 0 at a sample that is not clamped."""
    _, G, _, _ = decoder.jets(X, q_n)
    det = np.linalg.det(np.eye(3)[None] + G)
    free = np.ones(det.shape, bool) if clamp is None else ~np.asarray(clamp, dtype=bool)
    return bool(np.any((det <= 0.0) & free))


def elastic_step(decoder, X, q_n, q_prev, lam, mu, rho0, B, dt, opts: GNOptions, clamp=None):
    """q_n -> q_{n+1}; returns (q_next, info, targets)."""
    target, _ = elastic_targets(decoder, X, q_n, q_prev, lam, mu, rho0, B, dt, clamp)
    q_next, info = invert(decoder, X, target, q_n, opts)
    if inverted(decoder, X, q_n, clamp):
        info.flags |= INVERTED
    return q_next, info, target
