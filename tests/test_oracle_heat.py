"""Pins for the heat-equation pieces of the oracle and for the three-stage
latent step driven by an analytic decoder (no GPU).

The pins come from the mathematics of the paper's PDEs, not from the oracle:
* the explicit FD scheme maps each discrete sine mode to itself with a
  known amplification factor (exact to rounding);
* the continuous sine-mode solution is reached within the scheme's
  O(dx^2 + dt) truncation error;
* with a decoder that spans exactly the sine modes, one latent step is
  q_k -> (1 - dt nu k^2 pi^2) q_k, because the least-squares projection of
  an element of the span is exact.
"""
import numpy as np
import pytest

from oracle import heat, step
from oracle.inversion import GNOptions


def test_fd1d_discrete_mode_exact():
    n = 101
    dx = 1.0 / (n - 1)
    x = np.arange(n) * dx
    nu, dt, steps = 0.7, 0.3 * dx * dx / 0.7, 37
    for k in (1, 4, 9):
        u0 = np.sin(k * np.pi * x)
        lam = 1.0 - 4.0 * nu * dt / dx ** 2 * np.sin(k * np.pi * dx / 2) ** 2
        u = heat.fd_heat1d(u0, nu, dx, dt, steps)
        np.testing.assert_allclose(u, lam ** steps * u0, rtol=0, atol=1e-13)


def test_fd2d_discrete_mode_exact():
    n = 33
    dx = 1.0 / (n - 1)
    x = np.arange(n) * dx
    nu = 0.4
    dt = 0.2 * dx * dx / nu
    X, Y = np.meshgrid(x, x, indexing="ij")
    for k, l in ((1, 1), (2, 3), (5, 1)):
        u0 = np.sin(k * np.pi * X) * np.sin(l * np.pi * Y)
        rr = nu * dt / dx ** 2
        lam = 1.0 - 4.0 * rr * (np.sin(k * np.pi * dx / 2) ** 2 + np.sin(l * np.pi * dx / 2) ** 2)
        u = heat.fd_heat2d(u0, nu, dx, dt, 25)
        np.testing.assert_allclose(u, lam ** 25 * u0, rtol=0, atol=1e-13)


def test_fd1d_converges_to_continuous_modes():
    a = np.array([0.8, -0.5, 0.3])
    nu, T = 0.5, 0.01
    errs = []
    for n in (51, 101, 201):
        dx = 1.0 / (n - 1)
        dt = 0.25 * dx * dx / nu
        steps = int(round(T / dt))
        dt = T / steps
        x = np.arange(n) * dx
        u = heat.fd_heat1d(heat.heat1d_modes(a, nu, 0.0, x), nu, dx, dt, steps)
        errs.append(np.abs(u - heat.heat1d_modes(a, nu, T, x)).max())
    # Second order in dx at fixed dt/dx^2: halving dx quarters the error.
    assert errs[1] < errs[0] / 3.5 and errs[2] < errs[1] / 3.5


def test_fd2d_zero_boundary_and_symmetry():
    g = np.random.Generator(np.random.PCG64(3))
    u0 = g.uniform(-1, 1, size=(17, 17))
    u = heat.fd_heat2d(u0, 1.0, 1 / 16, 0.2 / 256, 10)
    assert np.all(u[0] == 0) and np.all(u[-1] == 0) and np.all(u[:, 0] == 0) and np.all(u[:, -1] == 0)
    # The scheme commutes with transposition of the grid.
    np.testing.assert_allclose(heat.fd_heat2d(u0.T, 1.0, 1 / 16, 0.2 / 256, 10), u.T, atol=1e-15)


def test_rom_targets_and_clamp():
    g = np.array([[1.0], [2.0], [3.0]])
    lap = np.array([[-4.0], [1.0], [0.5]])
    f = heat.rom_heat_targets(g, lap, 0.5, 0.1, clamp=np.array([0, 1, 0], dtype=np.uint8))
    np.testing.assert_allclose(f[:, 0], [1.0 - 0.2, 0.0, 3.0 + 0.025])


@pytest.mark.parametrize("r,n_samples", [(3, 3), (3, 20), (5, 11)])
def test_sine_decoder_one_step_exact(r, n_samples):
    dec = heat.SineModes1D(r)
    y = (np.arange(1, n_samples + 1) / (n_samples + 1.0))[:, None]
    q = np.array([0.9, -0.4, 0.25, 0.1, -0.05])[:r]
    nu, dt = 0.5, 1e-3
    for linearized in (False, True):
        q1, info, _ = step.heat_step(dec, y, q, nu, dt, GNOptions(max_iter=5, linearized=linearized))
        k = np.arange(1, r + 1)
        np.testing.assert_allclose(q1, (1 - dt * nu * (k * np.pi) ** 2) * q, rtol=1e-12, atol=1e-14)
        assert info.flags == 0


def test_sine_decoder_rollout_matches_closed_form():
    # Forward Euler in the latent coordinates: error O(dt) after T = 0.02.
    a = np.array([0.7, -0.3, 0.2])
    dec = heat.SineModes1D(3)
    y = (np.arange(1, 21) / 21.0)[:, None]
    nu, T = 0.5, 0.02
    xs = np.linspace(0, 1, 41)
    errs = []
    for steps in (200, 400):
        qs, _ = step.heat_rollout(dec, y, a, nu, T / steps, steps, GNOptions(max_iter=3))
        u = dec.value(xs[:, None], qs[-1])[:, 0]
        errs.append(np.abs(u - heat.heat1d_modes(a, nu, T, xs)).max())
    assert errs[0] < 5e-3
    assert 1.8 < errs[0] / errs[1] < 2.2


def test_sine2d_decoder_step_exact():
    dec = heat.SineModes2D(2, 2)
    g = np.random.Generator(np.random.PCG64(5))
    y = g.uniform(0.05, 0.95, size=(30, 2))
    q = g.uniform(-1, 1, size=4)
    nu, dt = 0.3, 2e-4
    q1, info, _ = step.heat_step(dec, y, q, nu, dt, GNOptions())
    lam = np.array([1 + 1, 1 + 4, 4 + 1, 4 + 4]) * np.pi ** 2
    np.testing.assert_allclose(q1, (1 - dt * nu * lam) * q, rtol=1e-12, atol=1e-14)


def test_energy_balance_1d_modes():
    # d/dt int_{x1}^{x2} u dx = nu (u_x(x2) - u_x(x1)) for the closed form,
    # and the FD solution satisfies it to discretisation accuracy.
    a = np.array([0.8, -0.5, 0.3])
    nu, x1, x2 = 0.5, 0.396, 0.526
    n = 2001
    dx = 1.0 / (n - 1)
    x = np.arange(n) * dx
    dt = 0.2 * dx * dx / nu
    steps = 200
    u0 = heat.heat1d_modes(a, nu, 0.0, x)
    u1 = heat.fd_heat1d(u0, nu, dx, dt, steps)
    sel = (x >= x1) & (x <= x2)

    def integral(u):
        return np.trapezoid(u[sel], x[sel])

    def flux(u):
        i1, i2 = np.where(sel)[0][[0, -1]]
        return nu * ((u[i2 + 1] - u[i2 - 1]) - (u[i1 + 1] - u[i1 - 1])) / (2 * dx)

    lhs = (integral(u1) - integral(u0)) / (steps * dt)
    mid = heat.fd_heat1d(u0, nu, dx, dt, steps // 2)
    assert abs(lhs - flux(mid)) < 1e-3 * max(1.0, abs(lhs))


def test_encoder_guess_of_sine_modes_is_the_modal_euler_update():
    """With the analytic sine-mode decoder and the least-squares projection
    onto its modes as the encoder, the guess is the exact modal forward-Euler
    update q_k (1 - dt nu (k pi)^2)."""
    from oracle.step import encoder_guess
    dec = heat.SineModes1D(4)
    x = np.linspace(0.0, 1.0, 101)[:, None]
    B, _ = dec._basis(x)
    P = np.linalg.pinv(B)
    q = np.array([0.7, -0.4, 0.25, 0.1])
    nu, dt = 0.5, 1e-3
    guess = encoder_guess(dec, lambda f: f @ P.T, x, q, nu, dt)
    k = np.arange(1, 5)
    np.testing.assert_allclose(guess, q * (1.0 - dt * nu * (k * np.pi) ** 2), rtol=1e-12, atol=1e-14)
