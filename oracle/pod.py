"""Proper orthogonal decomposition baseline in FP64 (test infrastructure only).

Sec. "Comparison with Prior Approaches": POD represents the discretised field
by a linear basis, u = U q with U of size (P d) x r, built from a singular
value decomposition of the discretised training data; inference (step 1) and
inversion (step 3) use U in place of the decoder, and the PDE time stepping
(step 2) is the method's own.  Readings: the basis is the r leading left
singular vectors of the snapshot matrix whose columns are the training
snapshots, without centring (u = U q, as the section writes it); for the
heat equation the basis is known only at the grid nodes, so the Laplacian
that step 2 needs is the full-order model's 5-point stencil applied to the
basis vectors (boundary nodes carry none).

``PODDecoder`` has the decoder interface of ``oracle.step`` (value,
value_jac_q, laplacian), with sample "points" given as node indices into the
flattened (nx, ny) grid, so ``oracle.step.heat_step`` runs it unchanged.
"""
from __future__ import annotations

import numpy as np


def pod_basis(snaps: np.ndarray, r: int) -> np.ndarray:
    """U [P, r]: the leading r left singular vectors of the snapshot matrix
    whose columns are the rows of snaps [N, P]."""
    X = np.asarray(snaps, dtype=np.float64).reshape(snaps.shape[0], -1).T  # [P, N]
    U, _, _ = np.linalg.svd(X, full_matrices=False)
    return U[:, :r].copy()


def grid_laplacian(field: np.ndarray, nx: int, ny: int, dx: float) -> np.ndarray:
    """5-point Laplacian of the fields [P, k] on the (nx, ny) grid (index
    i_x * ny + i_y); boundary nodes get 0."""
    f = np.asarray(field, dtype=np.float64).reshape(nx, ny, -1)
    lap = np.zeros_like(f)
    lap[1:-1, 1:-1] = (f[:-2, 1:-1] + f[2:, 1:-1] + f[1:-1, :-2] + f[1:-1, 2:] - 4.0 * f[1:-1, 1:-1]) / (dx * dx)
    return lap.reshape(nx * ny, -1)


class PODDecoder:
    """g(node, q) = U[node] q and its grid Laplacian (L_h U)[node] q."""

    def __init__(self, U: np.ndarray, nx: int, ny: int, dx: float):
        self.U = np.asarray(U, dtype=np.float64)
        self.LU = grid_laplacian(self.U, nx, ny, dx)
        self.r = self.U.shape[1]

    def value(self, y, q):
        return (self.U[np.asarray(y)] @ np.asarray(q, dtype=np.float64)).reshape(-1, 1)

    def value_jac_q(self, y, q):
        Uy = self.U[np.asarray(y)]
        return (Uy @ np.asarray(q, dtype=np.float64)).reshape(-1, 1), Uy.reshape(-1, 1, self.r).copy()

    def laplacian(self, y, q):
        return (self.LU[np.asarray(y)] @ np.asarray(q, dtype=np.float64)).reshape(-1, 1)

    def encode(self, field: np.ndarray) -> np.ndarray:
        """Latent of a full field [P] by orthogonal projection (U^T U = I)."""
        return self.U.T @ np.asarray(field, dtype=np.float64).ravel()

    def decode(self, q) -> np.ndarray:
        """The field [P] at every node."""
        return self.U @ np.asarray(q, dtype=np.float64)
