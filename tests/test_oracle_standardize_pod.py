"""Pins for the oracle's standardization fold (Sec. "Training Details") and
its POD baseline (Sec. "Comparison with Prior Approaches"), no GPU.

Standardization: a hand-worked example, affine equivariance of the moments,
and the fold checked through the networks themselves: the folded decoder
evaluated at physical points must equal u_std * g_s(x_s, q) + u_mean of the
standardized one, and the folded encoder at a physical field must equal the
standardized encoder at the standardized field (dense and convolutional).

POD: a snapshot matrix built with known singular vectors and values gives
that basis back (up to sign); with snapshots made of discrete sine modes of
the 5-point Laplacian (exact eigenvectors on the grid with zero boundary),
one POD heat step equals one full-order finite-difference step, which is the
modal Euler update of each coefficient."""
import numpy as np
import pytest

from oracle import heat, mlp, pod, step, train
from oracle.inversion import GNOptions
from workloads import rng, xavier_mlp


def test_standardization_worked_example():
    snaps = np.array([[1.0, 2.0], [3.0, 4.0]])
    nodes = np.array([[0.0, 10.0], [1.0, 10.0], [2.0, 13.0], [3.0, 15.0]])
    um, us, xm, xs = train.standardization(snaps, nodes)
    # values 1..4: mean 2.5, population variance (2.25 + 0.25) / 2 = 1.25
    assert um == pytest.approx(2.5, abs=1e-15)
    assert us == pytest.approx(np.sqrt(1.25), abs=1e-15)
    # x: 0..3 -> mean 1.5, variance 1.25; y: 10, 10, 13, 15 -> mean 12,
    # variance (4 + 4 + 1 + 9) / 4 = 4.5
    assert np.allclose(xm, [1.5, 12.0], atol=1e-15)
    assert np.allclose(xs, [np.sqrt(1.25), np.sqrt(4.5)], atol=1e-15)


def test_standardization_affine_equivariance():
    g = rng(1)
    snaps = g.normal(size=(7, 50))
    nodes = g.uniform(size=(50, 3))
    um, us, xm, xs = train.standardization(snaps, nodes)
    a, b = -2.5, 0.75
    um2, us2, xm2, xs2 = train.standardization(a * snaps + b, nodes * np.array([2.0, 3.0, 0.5]) + 1.0)
    assert um2 == pytest.approx(a * um + b, rel=1e-13)
    assert us2 == pytest.approx(abs(a) * us, rel=1e-13)
    assert np.allclose(xm2, xm * [2.0, 3.0, 0.5] + 1.0, rtol=1e-13)
    assert np.allclose(xs2, xs * [2.0, 3.0, 0.5], rtol=1e-13)


@pytest.mark.parametrize("m,d", [(2, 1), (3, 3)])
def test_fold_decoder_identity(m, d):
    g = rng(2)
    r, w = 4, 12
    dec = [(W.astype(np.float64), b.astype(np.float64)) for W, b in xavier_mlp(g, m, r, d, w, 3, 0.3)]
    enc = [(W.astype(np.float64), b.astype(np.float64)) for W, b in xavier_mlp(g, 20 * d, 0, r, 6, 1, 0.3)]
    stats = (0.37, 2.3, g.uniform(-1, 1, m), g.uniform(0.2, 3.0, m))
    fdec, _ = train.fold_standardization(dec, enc, stats, m)
    x = g.uniform(-2, 2, size=(40, m))
    for _ in range(3):
        q = g.uniform(-1, 1, r)
        ref = stats[1] * mlp.decode(dec, (x - stats[2]) / stats[3], q) + stats[0]
        assert np.abs(mlp.decode(fdec, x, q) - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_fold_dense_encoder_identity():
    g = rng(3)
    n_in, r = 30, 4
    dec = [(W.astype(np.float64), b.astype(np.float64)) for W, b in xavier_mlp(g, 2, r, 1, 8, 2, 0.3)]
    enc = [(W.astype(np.float64), b.astype(np.float64)) for W, b in xavier_mlp(g, n_in, 0, r, 10, 1, 0.3)]
    stats = (-0.8, 0.45, np.zeros(2), np.ones(2))
    _, fenc = train.fold_standardization(dec, enc, stats, 2)
    u = g.normal(size=(5, n_in)) * 0.5 - 0.8
    ref = train.encode(enc, (u - stats[0]) / stats[1])
    assert np.abs(train.encode(fenc, u) - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("d", [1, 3])
def test_fold_conv_encoder_identity(d):
    g = rng(4)
    n, r = 200, 4
    enc = [tuple(np.asarray(t, np.float64) for t in layer) for layer in train.conv_encoder_init(g, n, d, r, 16)]
    dec = [(W.astype(np.float64), b.astype(np.float64)) for W, b in xavier_mlp(g, 3, r, d, 8, 2, 0.3)]
    stats = (1.3, 0.6, np.zeros(3), np.ones(3))
    _, fenc = train.fold_standardization(dec, enc, stats, 3, enc_kind="conv")
    u = g.normal(size=(3, n * d)) * 0.6 + 1.3
    ref, _ = train.conv_encoder_forward(enc, (u - stats[0]) / stats[1], d)
    got, _ = train.conv_encoder_forward(fenc, u, d)
    assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_pod_basis_recovers_known_singular_vectors():
    g = rng(5)
    P, N, r = 60, 12, 4
    A, _ = np.linalg.qr(g.normal(size=(P, N)))
    B, _ = np.linalg.qr(g.normal(size=(N, N)))
    s = np.array([9.0, 5.0, 3.0, 2.0, 1e-1, 5e-2, 1e-2, 5e-3, 1e-3, 5e-4, 1e-4, 5e-5])
    X = A @ np.diag(s) @ B.T              # columns are snapshots
    U = pod.pod_basis(X.T, r)
    assert U.shape == (P, r)
    assert np.abs(U.T @ U - np.eye(r)).max() < 1e-13
    # each basis vector is the corresponding singular vector up to sign
    for k in range(r):
        assert abs(abs(U[:, k] @ A[:, k]) - 1.0) < 1e-12


def _sine_grid(nx, modes, coef):
    xs = np.arange(nx) / (nx - 1)
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    return sum(c * np.sin(k * np.pi * X) * np.sin(l * np.pi * Y) for c, (k, l) in zip(coef, modes))


@pytest.mark.parametrize("linearized", [True, False])
def test_pod_heat_step_on_sine_modes_is_the_fd_step(linearized):
    g = rng(6)
    nx = 21
    dx = 1.0 / (nx - 1)
    modes = [(1, 1), (2, 1), (1, 3), (4, 2), (3, 3)]
    snaps = np.stack([_sine_grid(nx, modes, g.uniform(-1, 1, len(modes))).ravel() for _ in range(12)])
    dec = pod.PODDecoder(pod.pod_basis(snaps, len(modes)), nx, nx, dx)
    coef = g.uniform(-1, 1, len(modes))
    u0 = _sine_grid(nx, modes, coef)
    q = dec.encode(u0)
    assert np.abs(dec.decode(q) - u0.ravel()).max() < 1e-13
    nu, dt = 0.6, 2e-4
    samples = g.choice(nx * nx, 40, replace=False)
    opts = GNOptions(max_iter=3, linearized=linearized, tol_step=1e-12)
    for n in range(1, 4):
        q, info, _ = step.heat_step(dec, samples, q, nu, dt, opts)
        assert info.flags == 0
        # full-order step and the discrete modal Euler update agree
        fd = heat.fd_heat2d(u0, nu, dx, dt, n)
        lam = [4.0 / dx ** 2 * (np.sin(k * np.pi * dx / 2) ** 2 + np.sin(l * np.pi * dx / 2) ** 2) for k, l in modes]
        modal = _sine_grid(nx, modes, [c * (1.0 - dt * nu * L) ** n for c, L in zip(coef, lam)])
        assert np.abs(fd - modal).max() < 1e-13
        assert np.abs(dec.decode(q) - fd.ravel()).max() < 1e-12


def test_pod_grid_laplacian_of_a_quadratic():
    # the 5-point stencil is exact on quadratics: Lap(x^2 + 3 y^2) = 8 inside
    nx = 9
    dx = 1.0 / (nx - 1)
    xs = np.arange(nx) * dx
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    lap = pod.grid_laplacian((X ** 2 + 3 * Y ** 2).reshape(-1, 1), nx, nx, dx).reshape(nx, nx)
    assert np.allclose(lap[1:-1, 1:-1], 8.0, atol=1e-10)
    assert np.all(lap[0] == 0) and np.all(lap[-1] == 0) and np.all(lap[:, 0] == 0) and np.all(lap[:, -1] == 0)
