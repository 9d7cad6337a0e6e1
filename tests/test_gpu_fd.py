"""The HIP full-order heat solver reproduces the oracle's FP64 finite-
difference solver bit for bit (same operations in the same order, no fused
multiply-add) in 1D and 2D, with scalar and per-node diffusivity (GPU)."""
import numpy as np
import pytest

from oracle import heat
from workloads import rng

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("per_node", [False, True])
def test_fd1d_bit_exact(cuda, per_node):
    import torch
    from paper_2206_02607_amd import crom
    g = rng(1)
    n, n_grid = 257, 3
    u0 = g.uniform(-1, 1, size=(n_grid, n))
    nu = g.uniform(0.1, 1.0, size=(n_grid, n) if per_node else n_grid)
    dx = 1.0 / (n - 1)
    dt = 0.2 * dx * dx
    u = torch.from_numpy(u0.copy()).to(cuda)
    crom.fd_heat(u, torch.from_numpy(np.ascontiguousarray(nu)).to(cuda), dx, dt, 37)
    for k in range(n_grid):
        ref = heat.fd_heat1d(u0[k], nu[k], dx, dt, 37)
        np.testing.assert_array_equal(u[k].cpu().numpy(), ref)


@pytest.mark.parametrize("per_node", [False, True])
def test_fd2d_bit_exact(cuda, per_node):
    import torch
    from paper_2206_02607_amd import crom
    g = rng(2)
    nx, ny, n_grid = 65, 48, 2
    u0 = g.uniform(-1, 1, size=(n_grid, nx, ny))
    nu = g.uniform(0.1, 1.0, size=(n_grid, nx, ny) if per_node else n_grid)
    dx = 1.0 / 63
    dt = 0.2 * dx * dx
    u = torch.from_numpy(u0.copy()).to(cuda)
    crom.fd_heat(u, torch.from_numpy(np.ascontiguousarray(nu)).to(cuda), dx, dt, 21)
    for k in range(n_grid):
        ref = heat.fd_heat2d(u0[k], nu[k], dx, dt, 21)
        np.testing.assert_array_equal(u[k].cpu().numpy(), ref)


def test_fd2d_256_grid_mode_decay(cuda):
    """256 x 256 grid (the 2D heat workload's size): a discrete sine mode
    decays by its exact amplification factor."""
    import torch
    from paper_2206_02607_amd import crom
    n = 256
    dx = 1.0 / (n - 1)
    x = np.arange(n) * dx
    X, Y = np.meshgrid(x, x, indexing="ij")
    mu = 0.7
    dt = 0.2 * dx * dx / mu
    u0 = np.sin(2 * np.pi * X) * np.sin(3 * np.pi * Y)
    u = torch.from_numpy(u0[None].copy()).to(cuda)
    crom.fd_heat(u, torch.tensor([mu], dtype=torch.float64), dx, dt, 100)
    r = mu * dt / dx ** 2
    lam = 1 - 4 * r * (np.sin(2 * np.pi * dx / 2) ** 2 + np.sin(3 * np.pi * dx / 2) ** 2)
    np.testing.assert_allclose(u[0].cpu().numpy(), lam ** 100 * u0, rtol=0, atol=1e-12)
