"""Pins for the network-inversion oracle (no GPU).

* Cholesky against a library SVD least-squares solve and against the
  defining identity L L^T = A;
* Gauss-Newton on a latent-linear decoder reaches the least-squares
  minimiser in one iteration (the residual is linear in q), and the
  linearised inversion is the same first step;
* the accepted line-search step satisfies the Armijo inequality and
  alpha = 1 is accepted on latent-linear problems;
* singular normal equations raise the SINGULAR flag and keep the iterate.
"""
import numpy as np

from oracle import inversion, mlp, step
from oracle.inversion import GNOptions
from workloads import rng


def _gen(seed):
    return np.random.Generator(np.random.PCG64(seed))


def test_cholesky_identity_and_solve():
    g = _gen(0)
    for n in (1, 3, 8, 16):
        J = g.normal(size=(3 * n + 2, n))
        A = J.T @ J
        L = inversion.cholesky(A)
        assert np.allclose(np.triu(L, 1), 0)
        np.testing.assert_allclose(L @ L.T, A, rtol=1e-13, atol=1e-12)
        rho = g.normal(size=3 * n + 2)
        x = inversion.chol_solve(L, J.T @ rho)
        ref = np.linalg.lstsq(J, rho, rcond=None)[0]
        np.testing.assert_allclose(x, ref, rtol=1e-10, atol=1e-12)


def test_cholesky_singular():
    A = np.diag([4.0, 0.0, 1.0])
    assert inversion.cholesky(A) is None
    B = np.ones((3, 3))
    assert inversion.cholesky(B) is None
    C = np.diag([1.0, np.nan])
    assert inversion.cholesky(C) is None


class LatentLinear:
    """g(y, q) = h(y) + B(y) q with a nonlinear h and B: the inversion
    residual is linear in q."""

    def __init__(self, r, d):
        self.r, self.d, self.m = r, d, 1

    def _hb(self, y):
        y = np.asarray(y, dtype=np.float64).reshape(-1)
        h = np.stack([np.cos(3 * y + o) for o in range(self.d)], axis=1)
        B = np.stack([np.stack([np.sin((k + 1) * np.pi * y + 0.3 * o) * (1 + y ** o) for k in range(self.r)], axis=1)
                      for o in range(self.d)], axis=1)
        return h, B

    def value(self, y, q):
        h, B = self._hb(y)
        return h + B @ q

    def value_jac_q(self, y, q):
        h, B = self._hb(y)
        return h + B @ q, B


def test_gn_one_step_exact_on_latent_linear():
    g = _gen(1)
    for r, d, S in ((3, 1, 20), (4, 2, 7), (8, 1, 40)):
        dec = LatentLinear(r, d)
        y = g.uniform(0, 1, size=(S, 1))
        target = g.normal(size=(S, d))
        q0 = g.normal(size=r)
        h, B = dec._hb(y)
        ref = np.linalg.lstsq(B.reshape(S * d, r), (target - h).ravel(), rcond=None)[0]
        q1, info = step.invert(dec, y, target, q0, GNOptions(max_iter=1))
        np.testing.assert_allclose(q1, ref, rtol=1e-10, atol=1e-12)
        assert info.iters == 1 and info.ls_evals == 1      # alpha = 1 accepted
        ql, infol = step.invert(dec, y, target, q0, GNOptions(linearized=True))
        np.testing.assert_allclose(ql, q1, rtol=1e-12, atol=1e-14)
        q5, info5 = step.invert(dec, y, target, q0, GNOptions(max_iter=5, tol_step=1e-8))
        np.testing.assert_allclose(q5, ref, rtol=1e-10, atol=1e-12)
        assert info5.flags == 0 and info5.iters == 1        # second GN step is ~0 -> stop
        np.testing.assert_allclose(info5.obj_last,
                                   0.5 * np.sum((target - dec.value(y, ref)) ** 2), rtol=1e-10)


def test_gn_affine_mlp_one_step():
    # An MLP held in the linear ELU branch is affine in q: one GN step is exact.
    # Its latent Jacobian is the same at every point, so d >= r keeps it full rank.
    g = _gen(2)
    m, r, d = 2, 3, 3
    sizes = [m + r, 9, 7, d]
    layers = []
    for i, (a, b) in enumerate(zip(sizes[:-1], sizes[1:])):
        layers.append((g.uniform(0.1, 1.0, size=(b, a)), g.uniform(0, 0.5, size=b) + (10.0 if i == 0 else 0)))
    dec = mlp.MLPDecoder(layers, m)
    y = g.uniform(0, 1, size=(12, m))
    q0 = g.uniform(0, 1, size=r)
    target = dec.value(y, g.uniform(0, 1, size=r)) + 0.01 * g.normal(size=(12, d))
    J = dec.value_jac_q(y, q0)[1].reshape(-1, r)
    ref = q0 + np.linalg.lstsq(J, (target - dec.value(y, q0)).ravel(), rcond=None)[0]
    q1, info = step.invert(dec, y, target, q0, GNOptions(max_iter=1))
    np.testing.assert_allclose(q1, ref, rtol=1e-9, atol=1e-11)


def test_line_search_armijo_and_shrink():
    # A decoder with strong curvature in q: the full Gauss-Newton step
    # overshoots from far away and the line search has to shrink.
    class Curved:
        r, d, m = 1, 1, 1

        def value(self, y, q):
            y = np.asarray(y).reshape(-1, 1)
            return np.arctan(8.0 * q[0]) * (1 + y)

        def value_jac_q(self, y, q):
            y = np.asarray(y).reshape(-1, 1)
            return self.value(y, q), ((8.0 / (1 + 64.0 * q[0] ** 2)) * (1 + y))[:, :, None]

    dec = Curved()
    y = np.linspace(0, 1, 5)[:, None]
    target = np.arctan(8.0 * 0.05) * (1 + y)
    q0 = np.array([2.0])
    opts = GNOptions(max_iter=1)
    q1, info = step.invert(dec, y, target, q0, opts)
    assert info.ls_evals > 1 and info.flags & inversion.MAXITER
    # Recompute the Armijo condition at the accepted point from first principles.
    g0, J0 = dec.value_jac_q(y, q0)
    rho = (target - g0).ravel()
    Jf = J0.reshape(-1, 1)
    delta = float((Jf.T @ rho)[0] / (Jf.T @ Jf)[0, 0])
    alpha = float((q1 - q0)[0] / delta)
    assert abs(alpha - 0.5 ** (info.ls_evals - 1)) < 1e-12
    phi0 = 0.5 * rho @ rho
    phi1 = 0.5 * np.sum((target - dec.value(y, q1)) ** 2)
    assert phi1 <= phi0 - 1e-4 * alpha * float(Jf.T @ rho) * delta
    # The previous trial (alpha * 2) violated it.
    qp = q0 + 2 * alpha * delta
    phip = 0.5 * np.sum((target - dec.value(y, qp)) ** 2)
    assert phip > phi0 - 1e-4 * 2 * alpha * float(Jf.T @ rho) * delta
    # Converges with enough iterations.
    qn, infon = step.invert(dec, y, target, q0, GNOptions(max_iter=30, tol_step=1e-12))
    np.testing.assert_allclose(qn, [0.05], rtol=1e-8)


def test_singular_keeps_iterate():
    class Flat:
        r, d, m = 2, 1, 1

        def value(self, y, q):
            return np.zeros((len(y), 1)) + q[0]

        def value_jac_q(self, y, q):
            J = np.zeros((len(y), 1, 2))
            J[:, 0, 0] = 1.0                              # column for q_2 is zero
            return self.value(y, q), J

    q0 = np.array([0.3, -0.2])
    q1, info = step.invert(Flat(), np.zeros((4, 1)), np.ones((4, 1)), q0, GNOptions())
    assert info.flags & inversion.SINGULAR
    np.testing.assert_array_equal(q1, q0)


def test_nonfinite_flag():
    class Bad:
        r, d, m = 1, 1, 1

        def value(self, y, q):
            return np.full((len(y), 1), np.nan)

        def value_jac_q(self, y, q):
            return self.value(y, q), np.ones((len(y), 1, 1))

    q1, info = step.invert(Bad(), np.zeros((3, 1)), np.ones((3, 1)), np.array([1.0]), GNOptions())
    assert info.flags & inversion.NONFINITE


# ---------------------------------------------------------------------------
# Gauss-Newton with a second candidate start (initial guess)
# ---------------------------------------------------------------------------

def _exp_model(g, N=30, r=3):
    """value(q) = exp(G q) (elementwise), a smooth nonlinear model whose
    Gauss-Newton from a far start needs many iterations."""
    G = g.uniform(-1, 1, size=(N, r))
    q_star = g.uniform(-1, 1, size=r)
    target = np.exp(G @ q_star)

    def value_fn(q):
        return np.exp(G @ q)

    def value_jac_fn(q):
        v = np.exp(G @ q)
        return v, v[:, None] * G

    return value_fn, value_jac_fn, target, q_star


def test_guess_better_start_is_used():
    g = rng(71)
    vf, vjf, target, q_star = _exp_model(g)
    q_n = q_star + 1.5
    opts = GNOptions(max_iter=3, tol_step=1e-12)
    plain, pinfo = inversion.gauss_newton(vf, vjf, target, q_n, opts)
    guess = q_star + 1e-3 * g.uniform(-1, 1, size=q_star.size)
    q, info, used = inversion.gauss_newton_from_guess(vf, vjf, target, q_n, guess, opts)
    ref, rinfo = inversion.gauss_newton(vf, vjf, target, guess, opts)
    assert used
    np.testing.assert_array_equal(q, ref)
    assert info.iters == rinfo.iters and info.ls_evals == rinfo.ls_evals
    r_n = target - vf(q_n)
    assert info.obj_first == 0.5 * float(r_n @ r_n)
    # from the far start three iterations do not get there; from the guess they do
    assert np.abs(q - q_star).max() < 1e-9 < np.abs(plain - q_star).max()


def test_guess_worse_start_changes_nothing():
    g = rng(72)
    vf, vjf, target, q_star = _exp_model(g)
    q_n = q_star + 0.05
    opts = GNOptions(max_iter=5, tol_step=1e-12)
    plain, pinfo = inversion.gauss_newton(vf, vjf, target, q_n, opts)
    q, info, used = inversion.gauss_newton_from_guess(vf, vjf, target, q_n, q_star + 2.0, opts)
    assert not used
    np.testing.assert_array_equal(q, plain)
    assert (info.iters, info.ls_evals, info.flags) == (pinfo.iters, pinfo.ls_evals, pinfo.flags)


def test_guess_ignored_when_linearised_or_stationary():
    g = rng(73)
    N, r = 20, 4
    G = g.normal(size=(N, r))
    t = g.normal(size=N)
    q_star = np.linalg.lstsq(G, t, rcond=None)[0]

    def vf(q):
        return G @ q

    def vjf(q):
        return G @ q, G

    lin = GNOptions(max_iter=1, linearized=True)
    q_n = q_star + 0.3
    q, info, used = inversion.gauss_newton_from_guess(vf, vjf, t, q_n, q_star, lin)
    ref, _ = inversion.gauss_newton(vf, vjf, t, q_n, lin)
    assert not used
    np.testing.assert_array_equal(q, ref)
    # q_n already the minimiser: the guess (no better anyway) is not evaluated
    q, info, used = inversion.gauss_newton_from_guess(vf, vjf, t, q_star, q_star + 1e-3, GNOptions())
    assert not used and info.iters == 0
    np.testing.assert_array_equal(q, q_star)


def test_guess_exact_minimiser_needs_no_iteration():
    """Latent-linear model: the exact least-squares solution as the guess is
    accepted and Gauss-Newton stops there at once."""
    g = rng(74)
    N, r = 25, 3
    G = g.normal(size=(N, r))
    t = g.normal(size=N)
    q_star = np.linalg.lstsq(G, t, rcond=None)[0]
    q, info, used = inversion.gauss_newton_from_guess(lambda q: G @ q, lambda q: (G @ q, G), t,
                                                      q_star + 1.0, q_star, GNOptions(tol_step=1e-10))
    assert used and info.iters == 0
    np.testing.assert_allclose(q, q_star, atol=1e-14)
