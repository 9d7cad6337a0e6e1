"""Heat equation pieces in FP64 (test infrastructure only).

* The reduced-order update at the integration samples (Sec. "Step 2: PDE
  Time-stepping", eqs. "discrete-time" and "time-integration"): the time
  derivative comes from the exact PDE, u_t = nu * Laplacian(u), evaluated with
  the decoder's own second derivatives (Sec. "Reduced-order Model" of the
  thermodynamics and image examples), and first-order explicit Euler advances
  it.  A sample flagged as clamped carries the Dirichlet value 0 instead.
* The full-order finite-difference solvers the method is judged against
  (Sec. "Thermodynamics / Full-order Model": 3-point Laplacian; Sec. "Image
  Processing / Full-order Model": 5-point Laplacian; forward Euler;
  zero Dirichlet boundary).
* Closed-form sine-mode solutions of the continuous problem.
"""
from __future__ import annotations

import numpy as np


def rom_heat_targets(g: np.ndarray, lap: np.ndarray, nu: float, dt: float,
                     clamp=None) -> np.ndarray:
    """f_{n+1}(y_j) = g(y_j, q_n) + dt * nu * Laplacian g(y_j, q_n)."""
    f = np.asarray(g, dtype=np.float64) + dt * nu * np.asarray(lap, dtype=np.float64)
    if clamp is not None:
        f = np.where(np.asarray(clamp, dtype=bool).reshape(f.shape[0], *([1] * (f.ndim - 1))),
                     0.0, f)
    return f


def fd_heat1d(u0: np.ndarray, nu, dx: float, dt: float, steps: int) -> np.ndarray:
    """Explicit Euler with the 3-point Laplacian on nodes x_i = i*dx; the two
    end nodes are held at 0.  ``nu`` may be a scalar or one value per node."""
    u = np.asarray(u0, dtype=np.float64).copy()
    u[0] = 0.0
    u[-1] = 0.0
    nu = np.broadcast_to(np.asarray(nu, dtype=np.float64), u.shape)
    for _ in range(steps):
        lap = np.zeros_like(u)
        lap[1:-1] = (u[:-2] + u[2:] - 2.0 * u[1:-1]) / (dx * dx)
        u = u + dt * nu * lap
        u[0] = 0.0
        u[-1] = 0.0
    return u


def fd_heat2d(u0: np.ndarray, nu, dx: float, dt: float, steps: int) -> np.ndarray:
    """Explicit Euler with the 5-point Laplacian on an (nx, ny) node array
    indexed [i_x, i_y] with equal spacing; boundary nodes are held at 0."""
    u = np.asarray(u0, dtype=np.float64).copy()
    u[0, :] = u[-1, :] = u[:, 0] = u[:, -1] = 0.0
    nu = np.broadcast_to(np.asarray(nu, dtype=np.float64), u.shape)
    for _ in range(steps):
        lap = np.zeros_like(u)
        lap[1:-1, 1:-1] = (u[:-2, 1:-1] + u[2:, 1:-1] + u[1:-1, :-2] + u[1:-1, 2:]
                           - 4.0 * u[1:-1, 1:-1]) / (dx * dx)
        u = u + dt * nu * lap
        u[0, :] = u[-1, :] = u[:, 0] = u[:, -1] = 0.0
    return u


def heat1d_modes(a: np.ndarray, nu: float, t: float, x: np.ndarray) -> np.ndarray:
    """sum_k a_k exp(-nu k^2 pi^2 t) sin(k pi x), k = 1..len(a)."""
    x = np.asarray(x, dtype=np.float64).ravel()
    k = np.arange(1, len(a) + 1)
    return (np.asarray(a)[None, :] * np.exp(-nu * (k * np.pi) ** 2 * t)[None, :]
            * np.sin(np.pi * x[:, None] * k[None, :])).sum(axis=1)


def heat2d_modes(a: np.ndarray, nu: float, t: float, xy: np.ndarray) -> np.ndarray:
    """sum_{k,l} a_kl exp(-nu (k^2 + l^2) pi^2 t) sin(k pi x) sin(l pi y)."""
    xy = np.asarray(xy, dtype=np.float64)
    K, Lm = a.shape
    out = np.zeros(xy.shape[0])
    for k in range(1, K + 1):
        for l in range(1, Lm + 1):
            out += (a[k - 1, l - 1] * np.exp(-nu * (k * k + l * l) * np.pi ** 2 * t)
                    * np.sin(k * np.pi * xy[:, 0]) * np.sin(l * np.pi * xy[:, 1]))
    return out


class SineModes1D:
    """Analytic decoder g(x, q) = sum_k q_k sin(k pi x): a stand-in for the
    network that lets the step and inversion logic be checked on its own."""

    def __init__(self, r: int):
        self.r = r
        self.m = 1
        self.d = 1

    def _basis(self, y):
        y = np.asarray(y, dtype=np.float64).reshape(-1)
        k = np.arange(1, self.r + 1)
        return np.sin(np.pi * y[:, None] * k[None, :]), -(np.pi * k[None, :]) ** 2

    def value(self, y, q):
        B, _ = self._basis(y)
        return (B @ np.asarray(q, dtype=np.float64))[:, None]

    def value_jac_q(self, y, q):
        B, _ = self._basis(y)
        return (B @ q)[:, None], B[:, None, :]

    def laplacian(self, y, q):
        B, lam = self._basis(y)
        return ((B * lam) @ np.asarray(q, dtype=np.float64))[:, None]


class SineModes2D:
    """g(x, y, q) = sum_{k,l} q_{(k,l)} sin(k pi x) sin(l pi y), q row-major over (k, l)."""

    def __init__(self, K: int, L: int):
        self.K, self.L = K, L
        self.r = K * L
        self.m = 2
        self.d = 1

    def _basis(self, y):
        y = np.asarray(y, dtype=np.float64)
        cols, lams = [], []
        for k in range(1, self.K + 1):
            for l in range(1, self.L + 1):
                cols.append(np.sin(k * np.pi * y[:, 0]) * np.sin(l * np.pi * y[:, 1]))
                lams.append(-(k * k + l * l) * np.pi ** 2)
        return np.stack(cols, axis=1), np.array(lams)[None, :]

    def value(self, y, q):
        B, _ = self._basis(y)
        return (B @ np.asarray(q, dtype=np.float64))[:, None]

    def value_jac_q(self, y, q):
        B, _ = self._basis(y)
        return (B @ q)[:, None], B[:, None, :]

    def laplacian(self, y, q):
        B, lam = self._basis(y)
        return ((B * lam) @ np.asarray(q, dtype=np.float64))[:, None]
