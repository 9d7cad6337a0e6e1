"""Pins for the neo-Hookean oracle (no GPU): the stress against the textbook
energy, the stress derivative against finite differences of the stress, the
small-strain limit (linear elasticity), the divergence through the Hessian
against a finite-difference divergence of the stress field of an analytic
displacement, free fall, the tangent-space velocity with a latent-linear
decoder whose derivatives are closed forms, and the projection step."""
import numpy as np
import pytest

from oracle import elastic, mlp
from oracle.inversion import GNOptions
from workloads import rng, xavier_mlp

LAM, MU, RHO0 = 1e4, 4e3, 1000.0
B = np.array([0.0, 0.0, -9.81])


def _rand_F(g, scale=0.1):
    return np.eye(3) + scale * g.uniform(-1, 1, size=(3, 3))


def test_stress_vanishes_at_identity():
    assert np.abs(elastic.pk1(np.eye(3), LAM, MU)).max() == 0.0


def test_stress_is_energy_gradient():
    g = rng(1)
    F = _rand_F(g)
    P = elastic.pk1(F, LAM, MU)
    h = 1e-6
    fd = np.zeros((3, 3))
    for k in range(3):
        for l in range(3):
            E = np.zeros((3, 3))
            E[k, l] = h
            fd[k, l] = (elastic.energy(F + E, LAM, MU) - elastic.energy(F - E, LAM, MU)) / (2 * h)
    np.testing.assert_allclose(P, fd, rtol=1e-6, atol=1e-6 * np.abs(P).max())


def test_stress_derivative_is_fd_of_stress():
    g = rng(2)
    F = _rand_F(g, 0.2)
    A = elastic.dpk1(F, LAM, MU)
    h = 1e-6
    for k in range(3):
        for l in range(3):
            E = np.zeros((3, 3))
            E[k, l] = h
            fd = (elastic.pk1(F + E, LAM, MU) - elastic.pk1(F - E, LAM, MU)) / (2 * h)
            np.testing.assert_allclose(A[:, :, k, l], fd, rtol=1e-6, atol=1e-6 * np.abs(A).max())


def test_small_strain_limit_is_linear_elasticity():
    g = rng(3)
    G = g.uniform(-1, 1, size=(3, 3))
    lin = MU * (G + G.T) + LAM * np.trace(G) * np.eye(3)
    errs = []
    for eps in (1e-2, 1e-3):
        P = elastic.pk1(np.eye(3) + eps * G, LAM, MU)
        errs.append(np.abs(P - eps * lin).max())
    # the remainder is second order in the strain
    assert errs[1] < errs[0] / 50


def _field(X):
    """An analytic displacement and its exact gradient and Hessian
    (hess[k, l, j] = d2u_k / dX_l dX_j)."""
    x, y, z = X
    u = 0.02 * np.array([np.sin(x) * y, x * x * z, np.cos(y) * z * z])
    G = 0.02 * np.array([[np.cos(x) * y, np.sin(x), 0.0],
                         [2 * x * z, 0.0, x * x],
                         [0.0, -np.sin(y) * z * z, 2 * np.cos(y) * z]])
    H = np.zeros((3, 3, 3))
    H[0] = 0.02 * np.array([[-np.sin(x) * y, np.cos(x), 0], [np.cos(x), 0, 0], [0, 0, 0]])
    H[1] = 0.02 * np.array([[2 * z, 0, 2 * x], [0, 0, 0], [2 * x, 0, 0]])
    H[2] = 0.02 * np.array([[0, 0, 0], [0, -np.cos(y) * z * z, -2 * np.sin(y) * z],
                            [0, -2 * np.sin(y) * z, 2 * np.cos(y)]])
    return u, G, H


def test_divergence_matches_fd_of_stress_field():
    X = np.array([0.7, 0.4, 0.9])
    _, G, H = _field(X)
    got = elastic.div_pk1((np.eye(3) + G)[None], H[None], LAM, MU)[0]
    h = 1e-5
    fd = np.zeros(3)
    for j in range(3):
        e = np.zeros(3)
        e[j] = h
        Pp = elastic.pk1(np.eye(3) + _field(X + e)[1], LAM, MU)
        Pm = elastic.pk1(np.eye(3) + _field(X - e)[1], LAM, MU)
        fd += (Pp[:, j] - Pm[:, j]) / (2 * h)
    np.testing.assert_allclose(got, fd, rtol=1e-6, atol=1e-6 * np.abs(fd).max())


def test_free_fall_targets():
    """A decoder that is identically zero: F = I, div P = 0 and J = 0, so one
    step from rest moves every sample by dt^2 B."""
    g = rng(4)
    layers = xavier_mlp(g, 3, 16, 3, 32, 3)
    layers[-1] = (np.zeros_like(layers[-1][0]), np.zeros_like(layers[-1][1]))
    dec = mlp.MLPDecoder(layers, 3)
    X = g.uniform(0, 1, size=(7, 3))
    q = g.uniform(-1, 1, size=16)
    dt = 1e-3
    tgt, inc = elastic.elastic_targets(dec, X, q, q - 0.1, LAM, MU, RHO0, B, dt)
    np.testing.assert_allclose(tgt, np.tile(dt * dt * B, (7, 1)), rtol=1e-14, atol=0)
    np.testing.assert_allclose(inc, tgt, rtol=0, atol=0)


class _PolyDecoder:
    """u_k(X, q) = sum_r q_r psi_{k r}(X) with quadratic psi: closed-form
    value, gradient, Hessian and latent Jacobian."""

    def __init__(self, g, r=4):
        self.r, self.m, self.d = r, 3, 3
        self.c = 0.01 * g.uniform(-1, 1, size=(3, r))
        self.a = 0.01 * g.uniform(-1, 1, size=(3, r, 3))
        b = 0.01 * g.uniform(-1, 1, size=(3, r, 3, 3))
        self.b = 0.5 * (b + np.swapaxes(b, -1, -2))  # psi = c + a.X + X.b.X

    def psi(self, X):
        return (self.c[None] + np.einsum("krl,sl->skr", self.a, X)
                + np.einsum("sl,krlj,sj->skr", X, self.b, X))

    def jets(self, X, q):
        Jq = self.psi(X)
        u = Jq @ q
        dpsi = self.a[None] + 2 * np.einsum("krlj,sj->skrl", self.b, X)
        G = np.einsum("skrl,r->skl", dpsi, q)
        H = np.broadcast_to(2 * np.einsum("krlj,r->klj", self.b, q), (X.shape[0], 3, 3, 3)).copy()
        return u, G, H, Jq

    def value(self, X, q):
        return self.jets(X, q)[0]

    def value_jac_q(self, X, q):
        u, _, _, J = self.jets(X, q)
        return u, J


def test_targets_with_closed_form_decoder():
    """u+ = u + dt (J qdot + dt (div P / rho0 + B)), with the divergence taken
    by finite differences of the stress field and J the closed-form psi."""
    g = rng(5)
    dec = _PolyDecoder(g)
    X = g.uniform(0, 1, size=(5, 3))
    q_n = g.uniform(-1, 1, size=dec.r)
    q_prev = q_n - 0.05 * g.uniform(-1, 1, size=dec.r)
    dt = 1e-3
    tgt, inc = elastic.elastic_targets(dec, X, q_n, q_prev, LAM, MU, RHO0, B, dt)
    u, _, _, Jq = dec.jets(X, q_n)
    h = 1e-5
    for s in range(X.shape[0]):
        div = np.zeros(3)
        for j in range(3):
            e = np.zeros(3)
            e[j] = h
            Pp = elastic.pk1(np.eye(3) + dec.jets((X[s] + e)[None], q_n)[1][0], LAM, MU)
            Pm = elastic.pk1(np.eye(3) + dec.jets((X[s] - e)[None], q_n)[1][0], LAM, MU)
            div += (Pp[:, j] - Pm[:, j]) / (2 * h)
        v = Jq[s] @ ((q_n - q_prev) / dt)
        expect = u[s] + dt * (v + dt * (div / RHO0 + B))
        np.testing.assert_allclose(tgt[s], expect, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(inc[s], tgt[s] - u[s], rtol=1e-9, atol=1e-15)


def test_clamped_samples_target_zero():
    g = rng(6)
    dec = _PolyDecoder(g)
    X = g.uniform(0, 1, size=(6, 3))
    q = g.uniform(-1, 1, size=dec.r)
    clamp = np.array([1, 0, 1, 0, 0, 1], dtype=np.uint8)
    tgt, inc = elastic.elastic_targets(dec, X, q, None, LAM, MU, RHO0, B, 1e-3, clamp)
    assert np.all(tgt[clamp == 1] == 0.0)
    u = dec.value(X, q)
    np.testing.assert_array_equal(inc[clamp == 1], -u[clamp == 1])


@pytest.mark.parametrize("linearized", [True, False])
def test_step_is_least_squares_projection(linearized):
    """Latent-linear decoder: the step lands on the least-squares projection
    of the targets (all three components of every sample)."""
    g = rng(7)
    dec = _PolyDecoder(g, r=4)
    X = g.uniform(0, 1, size=(9, 3))
    q_n = g.uniform(-1, 1, size=dec.r)
    opts = GNOptions(max_iter=5, linearized=linearized, tol_step=1e-12)
    q1, info, tgt = elastic.elastic_step(dec, X, q_n, None, LAM, MU, RHO0, B, 1e-3, opts)
    Jq = dec.jets(X, q_n)[3].reshape(-1, dec.r)
    ls = np.linalg.lstsq(Jq, tgt.ravel(), rcond=None)[0]
    np.testing.assert_allclose(q1, ls, rtol=1e-9, atol=1e-12)


class _StretchDecoder:
    """u(X, q) = (c + q_0) X_1 e_1: F = diag(1 + c + q_0, 1, 1) everywhere,
    det F = 1 + c + q_0 in closed form; zero Hessian."""

    def __init__(self, c, r=2):
        self.c, self.r = c, r

    def jets(self, X, q):
        X = np.asarray(X, dtype=np.float64)
        S = len(X)
        s = self.c + q[0]
        u = np.zeros((S, 3))
        u[:, 0] = s * X[:, 0]
        G = np.zeros((S, 3, 3))
        G[:, 0, 0] = s
        Jq = np.zeros((S, 3, self.r))
        Jq[:, 0, 0] = X[:, 0]
        return u, G, np.zeros((S, 3, 3, 3)), Jq

    def value(self, X, q):
        return self.jets(X, q)[0]

    def value_jac_q(self, X, q):
        u, _, _, J = self.jets(X, q)
        return u, J


@pytest.mark.parametrize("c,flag", [(-2.0, True), (-1.0, True), (-0.5, False), (0.3, False)])
def test_inverted_flag_follows_det_F(c, flag):
    """det F = 1 + c: at or below zero the step reports INVERTED (with
    NONFINITE from ln J, q stays at q_n); above zero it does not."""
    from oracle.inversion import INVERTED, NONFINITE
    g = rng(8)
    dec = _StretchDecoder(c)
    X = g.uniform(0.1, 1, size=(5, 3))
    q_n = np.zeros(dec.r)
    q1, info, _ = elastic.elastic_step(dec, X, q_n, None, LAM, MU, RHO0, B, 1e-3, GNOptions(max_iter=3))
    assert bool(info.flags & INVERTED) == flag
    if flag:
        assert info.flags & NONFINITE and np.array_equal(q1, q_n)
    # clamped samples do not use the stress: inverting only there is no flag
    clamp = np.ones(5, np.uint8)
    _, info, _ = elastic.elastic_step(dec, X, q_n, None, LAM, MU, RHO0, B, 1e-3, GNOptions(max_iter=3), clamp)
    assert not info.flags & INVERTED
