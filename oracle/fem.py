"""Corotated linear elasticity with finite-element forces at the integration
samples, in FP64 (test infrastructure only).

Sec. "Solid Mechanics" of the appendix: the displacement u(X, t) = g(X, q(t))
gives the deformed positions x = X + u of mesh vertices; the elastic force on
a sample vertex is the sum of the forces of the linear tetrahedra incident on
it, and the deformation gradient of each tetrahedron comes from the
finite-element linear basis (the numerical gradient of Sec. "Network
Gradients via Numerical Differentiation"), not from the network's x-derivative.
The decoder is therefore evaluated at the samples' one-ring: every vertex of
every tetrahedron incident on a sample.

Per tetrahedron (Sec. "Full-order Model" of the appendix):
* D_m = [X_1 - X_4, X_2 - X_4, X_3 - X_4], D_s the same from the deformed
  positions, F = D_s D_m^-1;
* the first Piola-Kirchhoff stress of corotated linear elasticity,
  P(F) = 2 mu (F - R) + lam tr(R^T F - I) R, with R the rotation of the
  polar decomposition F = R S;
* vertex forces [f_1 f_2 f_3] = -(1/6) |det D_m| P(F) D_m^-T, f_4 = -(f_1 +
  f_2 + f_3).

Readings:
* the printed stress squares the trace; that form is not the derivative of
  the corotated energy and is not linear in the strain.  The stress here is
  the derivative of Psi(F) = mu |F - R|^2 + lam/2 tr(R^T F - I)^2 (the energy
  of the cited course notes), which is what the tests pin; in the paper's own
  experiment lam = 0 and both forms agree;
* R is the proper rotation (det R = +1) of F when det F > 0; an inverted or
  flat tetrahedron (det F <= 0) has no such factor and its stress is NaN (the
  latent step then reports a non-finite instance);
* lumped mass: a vertex carries rho0 / 4 of the volume of each incident
  tetrahedron;
* time stepping as for the network-derivative elastic step: velocity from
  the tangent space, v_n = (dg/dq)(q_n - q_{n-1})/dt (at rest without a
  previous latent), symplectic Euler at the samples,
  v+ = v_n + dt (f / m + B), target u+ = u + dt v+; a clamped sample targets
  u+ = 0; the inversion projects the targets onto the decoder at the samples.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

from .inversion import INVERTED, GNOptions
from .step import invert


def rotation(F: np.ndarray) -> np.ndarray:
    """Rotation factor R of the polar decomposition F = R S for F [.., 3, 3]
    (R = U V^T from the singular value decomposition F = U Sigma V^T; NaN where
    det F <= 0)."""
    F = np.asarray(F, dtype=np.float64)
    U, _, Vt = np.linalg.svd(F)
    R = U @ Vt
    bad = np.linalg.det(F) <= 0
    return np.where(bad[..., None, None], np.nan, R)


def pk1(F: np.ndarray, lam: float, mu: float) -> np.ndarray:
    """Corotated first Piola-Kirchhoff stress P(F) [.., 3, 3]."""
    F = np.asarray(F, dtype=np.float64)
    R = rotation(F)
    tr = np.trace(np.swapaxes(R, -1, -2) @ F, axis1=-2, axis2=-1) - 3.0
    return 2.0 * mu * (F - R) + lam * tr[..., None, None] * R


def energy(F: np.ndarray, lam: float, mu: float) -> float:
    """Corotated energy density Psi(F) = mu |F - R|^2 + lam/2 tr(R^T F - I)^2."""
    F = np.asarray(F, dtype=np.float64)
    R = rotation(F)
    return float(mu * np.sum((F - R) ** 2) + 0.5 * lam * (np.trace(R.T @ F) - 3.0) ** 2)


def rest_shape(X: np.ndarray, tet) -> Tuple[np.ndarray, float]:
    """D_m [3, 3] (columns X_a - X_4) and the volume |det D_m| / 6 of one
    tetrahedron with vertex indices tet [4] into X [V, 3]."""
    X = np.asarray(X, dtype=np.float64)
    a, b, c, e = (int(v) for v in tet)
    Dm = np.stack([X[a] - X[e], X[b] - X[e], X[c] - X[e]], axis=1)
    return Dm, abs(np.linalg.det(Dm)) / 6.0


def deformation_gradient(x: np.ndarray, X: np.ndarray, tet) -> np.ndarray:
    """F = D_s D_m^-1 of one tetrahedron (x deformed, X rest positions)."""
    x = np.asarray(x, dtype=np.float64)
    a, b, c, e = (int(v) for v in tet)
    Ds = np.stack([x[a] - x[e], x[b] - x[e], x[c] - x[e]], axis=1)
    Dm, _ = rest_shape(X, tet)
    return Ds @ np.linalg.inv(Dm)


def tet_forces(x: np.ndarray, X: np.ndarray, tet, lam: float, mu: float) -> np.ndarray:
    """Forces [4, 3] on the four vertices of one tetrahedron."""
    Dm, vol = rest_shape(X, tet)
    F = deformation_gradient(x, X, tet)
    H = -vol * pk1(F, lam, mu) @ np.linalg.inv(Dm).T
    f = np.empty((4, 3))
    f[:3] = H.T
    f[3] = -H.sum(axis=1)
    return f


def tet_energy(x: np.ndarray, X: np.ndarray, tet, lam: float, mu: float) -> float:
    """Elastic energy vol * Psi(F) of one tetrahedron."""
    _, vol = rest_shape(X, tet)
    return vol * energy(deformation_gradient(x, X, tet), lam, mu)


def one_ring(tets: np.ndarray, samples) -> Tuple[List[np.ndarray], np.ndarray]:
    """For each sample vertex, the indices of the tetrahedra that contain it
    (ascending); and the sorted set of all vertices of those tetrahedra (the
    samples included)."""
    tets = np.asarray(tets)
    incident = [np.flatnonzero((tets == int(s)).any(axis=1)) for s in samples]
    verts = np.unique(np.concatenate([tets[t].ravel() for t in incident])) if incident else np.zeros(0, int)
    return incident, verts


def vertex_forces(x: np.ndarray, X: np.ndarray, tets: np.ndarray, samples, lam: float, mu: float) -> np.ndarray:
    """Elastic force [S, 3] on each sample vertex: the sum over its incident
    tetrahedra of that tetrahedron's force on it."""
    tets = np.asarray(tets)
    incident, _ = one_ring(tets, samples)
    out = np.zeros((len(samples), 3))
    for i, s in enumerate(samples):
        for t in incident[i]:
            corner = int(np.flatnonzero(tets[t] == int(s))[0])
            out[i] += tet_forces(x, X, tets[t], lam, mu)[corner]
    return out


def lumped_mass(X: np.ndarray, tets: np.ndarray, verts, rho0: float) -> np.ndarray:
    """rho0 / 4 of the volume of every tetrahedron incident on each vertex."""
    tets = np.asarray(tets)
    out = np.zeros(len(verts))
    for i, v in enumerate(verts):
        for t in np.flatnonzero((tets == int(v)).any(axis=1)):
            out[i] += rho0 * rest_shape(X, tets[t])[1] / 4.0
    return out


def fem_targets(decoder, X: np.ndarray, tets: np.ndarray, samples, q_n: np.ndarray, q_prev,
                lam: float, mu: float, rho0: float, B, dt: float, clamp=None):
    """Targets u+ [S, 3] at the sample vertices and the increments
    rho0 = u+ - u(q_n) [S, 3] (dt v+, or -u on a clamped sample).

    decoder.value(Y, q) -> [n, 3] displacements; decoder.value_jac_q(Y, q) ->
    (u [n, 3], du/dq [n, 3, r]).  X [V, 3] rest positions of the whole mesh,
    tets [T, 4] vertex indices, samples [S] vertex indices."""
    X = np.asarray(X, dtype=np.float64)
    samples = np.asarray(samples)
    _, ring = one_ring(tets, samples)
    x = np.full_like(X, np.nan)  # only the one-ring is decoded
    x[ring] = X[ring] + decoder.value(X[ring], q_n)
    f = vertex_forces(x, X, tets, samples, lam, mu)
    m = lumped_mass(X, tets, samples, rho0)
    u, Jq = decoder.value_jac_q(X[samples], q_n)
    qdot = np.zeros_like(q_n) if q_prev is None else (np.asarray(q_n) - np.asarray(q_prev)) / dt
    v = np.einsum("skr,r->sk", Jq, qdot)
    acc = f / m[:, None] + np.asarray(B, dtype=np.float64)[None, :]
    inc = dt * (v + dt * acc)
    if clamp is not None:
        c = np.asarray(clamp, dtype=bool)
        inc = np.where(c[:, None], -u, inc)
    return u + inc, inc


def inverted(decoder, X: np.ndarray, tets: np.ndarray, samples, q_n: np.ndarray, clamp=None) -> bool:
    """Whether a tetrahedron incident on a sample that is not clamped has
    det F <= 0 (no proper rotation factor: the corotated stress is
    undefined and the step reports INVERTED)."""
    X = np.asarray(X, dtype=np.float64)
    samples = np.asarray(samples)
    inc, ring = one_ring(tets, samples)
    x = np.full_like(X, np.nan)
    x[ring] = X[ring] + decoder.value(X[ring], q_n)
    free = np.ones(len(samples), bool) if clamp is None else ~np.asarray(clamp, dtype=bool)
    for s, ts in enumerate(inc):
        if free[s] and any(np.linalg.det(deformation_gradient(x, X, tets[t])) <= 0.0 for t in ts):
            return True
    return False


def fem_step(decoder, X, tets, samples, q_n, q_prev, lam, mu, rho0, B, dt, opts: GNOptions, clamp=None):
    """q_n -> q_{n+1}; returns (q_next, info, targets).  A sample's incident
    tetrahedron with det F <= 0 reports INVERTED (with NONFINITE from its NaN
    forces)."""
    target, _ = fem_targets(decoder, X, tets, samples, q_n, q_prev, lam, mu, rho0, B, dt, clamp)
    q_next, info = invert(decoder, np.asarray(X, dtype=np.float64)[np.asarray(samples)], target, q_n, opts)
    if inverted(decoder, X, tets, samples, q_n, clamp):
        info.flags |= INVERTED
    return q_next, info, target
