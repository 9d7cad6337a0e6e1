"""Pins for the corotated finite-element oracle (no GPU).

The rotation factor against a rotation built in closed form (Rodrigues) and
an SPD stretch; the stress against central differences of the corotated
energy, its rest state, frame indifference and small-strain limit (linear
elasticity); tetrahedron forces against central differences of the element
energy, zero net force and torque; vertex forces of a whole mesh against the
gradient of the total energy (which pins the corner bookkeeping and the
accumulation), and zero at interior vertices under an affine deformation; the
lumped masses against the box volume; the one-ring against a brute-force
scan; the targets for a translating decoder (free fall) and for a
latent-linear affine decoder whose velocity is a closed form; and the
projection step of that decoder against a least-squares solve."""
import numpy as np
import pytest

from oracle import fem
from oracle.inversion import GNOptions
from workloads import box_tet_mesh, rng

LAM, MU, RHO0 = 2.5e4, 1.2e4, 1000.0
B = np.array([0.0, 0.0, -9.81])


def _rodrigues(axis, angle):
    k = np.asarray(axis, dtype=np.float64) / np.linalg.norm(axis)
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + np.sin(angle) * K + (1 - np.cos(angle)) * K @ K


def _spd(g, scale=0.3):
    A = scale * g.uniform(-1, 1, size=(3, 3))
    return np.eye(3) + A @ A.T


def _mesh(g, n=(5, 4, 4), jitter=0.2):
    return box_tet_mesh(*n, 0.25, jitter, g)


def test_rotation_recovers_closed_form_factor():
    g = rng(1)
    for angle in (0.0, 0.3, 2.5, np.pi - 1e-3):
        Q = _rodrigues(g.normal(size=3), angle)
        S = _spd(g)
        R = fem.rotation(Q @ S)
        np.testing.assert_allclose(R, Q, atol=1e-12)
        assert abs(np.linalg.det(R) - 1.0) < 1e-12
        Sr = R.T @ (Q @ S)
        np.testing.assert_allclose(Sr, Sr.T, atol=1e-12)


def test_rotation_undefined_when_inverted():
    F = np.diag([1.0, 1.0, -0.5])
    assert np.isnan(fem.rotation(F)).all()
    assert np.isnan(fem.pk1(F, LAM, MU)).all()
    assert np.isnan(fem.rotation(np.diag([1.0, 1.0, 0.0]))).all()


@pytest.mark.parametrize("lam", [LAM, 0.0])
def test_stress_is_energy_gradient(lam):
    g = rng(2)
    F = _rodrigues(g.normal(size=3), 0.7) @ _spd(g)
    P = fem.pk1(F, lam, MU)
    h = 1e-6
    fd = np.zeros((3, 3))
    for k in range(3):
        for l in range(3):
            E = np.zeros((3, 3))
            E[k, l] = h
            fd[k, l] = (fem.energy(F + E, lam, MU) - fem.energy(F - E, lam, MU)) / (2 * h)
    np.testing.assert_allclose(P, fd, rtol=1e-6, atol=1e-7 * np.abs(P).max())


def test_stress_rest_state_and_frame_indifference():
    g = rng(3)
    Q = _rodrigues(g.normal(size=3), 1.1)
    assert np.abs(fem.pk1(Q, LAM, MU)).max() < 1e-9
    F = _rodrigues(g.normal(size=3), 0.4) @ _spd(g)
    np.testing.assert_allclose(fem.pk1(Q @ F, LAM, MU), Q @ fem.pk1(F, LAM, MU), rtol=1e-12,
                               atol=1e-9 * np.abs(fem.pk1(F, LAM, MU)).max())


def test_small_strain_limit_is_linear_elasticity():
    g = rng(4)
    G = g.uniform(-1, 1, size=(3, 3))
    lin = MU * (G + G.T) + LAM * np.trace(G) * np.eye(3)
    errs = []
    for eps in (1e-2, 1e-3):
        errs.append(np.abs(fem.pk1(np.eye(3) + eps * G, LAM, MU) - eps * lin).max())
    # the remainder is second order in the strain
    assert errs[1] < errs[0] / 50
    assert errs[1] < 1e-5 * np.abs(lin).max()


def test_tet_forces_are_energy_gradient():
    g = rng(5)
    X = g.uniform(0, 1, size=(4, 3))
    if np.linalg.det(np.stack([X[0] - X[3], X[1] - X[3], X[2] - X[3]], 1)) < 0:
        X[[0, 1]] = X[[1, 0]]
    tet = np.arange(4)
    x = (_rodrigues(g.normal(size=3), 0.8) @ _spd(g, 0.2) @ X.T).T + g.normal(size=3)
    f = fem.tet_forces(x, X, tet, LAM, MU)
    h = 1e-6
    fd = np.zeros((4, 3))
    for a in range(4):
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[a, k] += h
            xm[a, k] -= h
            fd[a, k] = -(fem.tet_energy(xp, X, tet, LAM, MU) - fem.tet_energy(xm, X, tet, LAM, MU)) / (2 * h)
    np.testing.assert_allclose(f, fd, rtol=1e-5, atol=1e-6 * np.abs(f).max())
    scale = np.abs(f).max()
    assert np.abs(f.sum(axis=0)).max() < 1e-12 * scale * 4
    assert np.abs(np.cross(x, f).sum(axis=0)).max() < 1e-11 * scale * np.abs(x).max() * 4


def test_vertex_forces_are_mesh_energy_gradient():
    g = rng(6)
    X, tets = _mesh(g)
    x = X.astype(np.float64) + 0.03 * g.uniform(-1, 1, size=X.shape)
    samples = np.array([0, 7, 26, 37, 52, 79])  # corners, edges, faces and interior vertices

    def total(xx):
        return sum(fem.tet_energy(xx, X, t, LAM, MU) for t in tets)

    f = fem.vertex_forces(x, X, tets, samples, LAM, MU)
    h = 1e-6
    for i, s in enumerate(samples):
        for k in range(3):
            xp, xm = x.copy(), x.copy()
            xp[s, k] += h
            xm[s, k] -= h
            fd = -(total(xp) - total(xm)) / (2 * h)
            assert abs(f[i, k] - fd) <= 1e-5 * np.abs(f).max(), (s, k, f[i, k], fd)


def test_affine_deformation_leaves_interior_vertices_unloaded():
    g = rng(7)
    nx, ny, nz = 5, 4, 4
    X, tets = _mesh(g, (nx, ny, nz))
    A = _rodrigues(g.normal(size=3), 0.5) @ _spd(g, 0.3)
    x = X.astype(np.float64) @ A.T + np.array([0.3, -0.1, 2.0])
    for t in tets[::17]:
        np.testing.assert_allclose(fem.deformation_gradient(x, X, t), A, atol=1e-12)
    idx = np.arange(nx * ny * nz)
    i, j, k = idx // (ny * nz), (idx // nz) % ny, idx % nz
    interior = idx[(i > 0) & (i < nx - 1) & (j > 0) & (j < ny - 1) & (k > 0) & (k < nz - 1)]
    boundary = idx[(i == 0) | (k == nz - 1)][:6]
    f_in = fem.vertex_forces(x, X, tets, interior, LAM, MU)
    f_bd = fem.vertex_forces(x, X, tets, boundary, LAM, MU)
    scale = np.abs(f_bd).max()
    assert scale > 1.0
    assert np.abs(f_in).max() < 1e-10 * scale


def test_lumped_mass_sums_to_box_mass():
    g = rng(8)
    nx, ny, nz, h = 5, 4, 4, 0.25
    X, tets = box_tet_mesh(nx, ny, nz, h, 0.2, g)
    m = fem.lumped_mass(X, tets, np.arange(nx * ny * nz), RHO0)
    box = (nx - 1) * (ny - 1) * (nz - 1) * h ** 3
    assert abs(m.sum() - RHO0 * box) < 1e-9 * RHO0 * box
    assert (m > 0).all()


def test_one_ring_brute_force():
    g = rng(9)
    X, tets = _mesh(g, (4, 3, 3))
    samples = [0, 5, 17, 35]
    inc, ring = fem.one_ring(tets, samples)
    want_ring = set()
    for i, s in enumerate(samples):
        want = [t for t in range(len(tets)) if s in set(int(v) for v in tets[t])]
        assert list(inc[i]) == want
        for t in want:
            want_ring.update(int(v) for v in tets[t])
    assert list(ring) == sorted(want_ring)
    # an interior vertex of the six-tetrahedra split touches 24 of them
    # (this mesh's interior vertices are (i*3 + 1)*3 + 1 for i = 1, 2); its
    # one-ring holds the 14 neighbours of the split and itself
    for v in (13, 22):
        inc_v, ring_v = fem.one_ring(tets, [v])
        assert len(inc_v[0]) == 24 and len(ring_v) == 15


class _Translate:
    """u(X, q) = c (no dependence on X or q)."""

    def __init__(self, c, r):
        self.c, self.r = np.asarray(c, dtype=np.float64), r

    def value(self, Y, q):
        return np.tile(self.c, (len(Y), 1))

    def value_jac_q(self, Y, q):
        return self.value(Y, q), np.zeros((len(Y), 3, self.r))


class _AffineLatent:
    """u(X, q) = (sum_k q_k E_k) X: latent-linear, F = I + sum_k q_k E_k on
    every tetrahedron, du/dq[:, :, k] = E_k X."""

    def __init__(self, E):
        self.E = np.asarray(E, dtype=np.float64)

    def value(self, Y, q):
        return np.asarray(Y, dtype=np.float64) @ np.einsum("k,kij->ij", q, self.E).T

    def value_jac_q(self, Y, q):
        J = np.einsum("kij,sj->sik", self.E, np.asarray(Y, dtype=np.float64))
        return self.value(Y, q), J


def test_targets_free_fall():
    g = rng(10)
    X, tets = _mesh(g)
    dec = _Translate([0.1, -0.2, 0.05], 4)
    samples = np.array([3, 30, 41, 70])
    dt = 1e-3
    t, inc = fem.fem_targets(dec, X, tets, samples, np.zeros(4), np.ones(4), LAM, MU, RHO0, B, dt)
    np.testing.assert_allclose(inc, np.tile(dt * dt * B, (4, 1)), atol=1e-18)
    np.testing.assert_allclose(t, np.tile(dec.c + dt * dt * B, (4, 1)), atol=1e-15)
    clamp = np.array([1, 0, 0, 1], np.uint8)
    t, inc = fem.fem_targets(dec, X, tets, samples, np.zeros(4), None, LAM, MU, RHO0, B, dt, clamp)
    np.testing.assert_allclose(t[[0, 3]], 0.0, atol=1e-18)
    np.testing.assert_allclose(inc[[0, 3]], -dec.c[None].repeat(2, 0), atol=1e-18)


def test_targets_affine_latent_decoder_interior():
    g = rng(11)
    nx, ny, nz = 5, 4, 4
    X, tets = _mesh(g, (nx, ny, nz))
    r = 3
    E = 0.05 * g.uniform(-1, 1, size=(r, 3, 3))
    dec = _AffineLatent(E)
    interior = np.array([(i * ny + j) * nz + k for i in (1, 2, 3) for j in (1, 2) for k in (1, 2)])
    q_n, q_prev = g.uniform(-1, 1, size=r), g.uniform(-1, 1, size=r)
    dt = 2e-3
    t, inc = fem.fem_targets(dec, X, tets, interior, q_n, q_prev, LAM, MU, RHO0, B, dt)
    Xs = X[interior].astype(np.float64)
    v = Xs @ np.einsum("k,kij->ij", (q_n - q_prev) / dt, E).T
    want = dt * (v + dt * B[None])  # interior forces vanish under the affine map
    np.testing.assert_allclose(inc, want, rtol=1e-9, atol=1e-12 * np.abs(want).max())
    np.testing.assert_allclose(t, dec.value(Xs, q_n) + want, rtol=1e-12, atol=1e-15)


def test_step_projection_of_affine_latent_decoder():
    g = rng(12)
    X, tets = _mesh(g)
    r = 3
    E = 0.05 * g.uniform(-1, 1, size=(r, 3, 3))
    dec = _AffineLatent(E)
    samples = np.array([1, 9, 22, 27, 40, 58, 63, 77])
    q_n = g.uniform(-1, 1, size=r)
    q1, info, target = fem.fem_step(dec, X, tets, samples, q_n, None, LAM, MU, RHO0, B, 1e-3,
                                    GNOptions(max_iter=5, tol_step=1e-13))
    _, J = dec.value_jac_q(X[samples], q_n)
    want = np.linalg.lstsq(J.reshape(-1, r), target.ravel(), rcond=None)[0]
    np.testing.assert_allclose(q1, want, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("scale,flag", [(-1.5, True), (-1.0, True), (-0.4, False)])
def test_inverted_flag_follows_det_F(scale, flag):
    """The affine decoder u = q_0 E X with E = e_1 e_1^T gives F = diag(1 +
    q_0, 1, 1) on every tetrahedron: det F = 1 + q_0 <= 0 reports INVERTED
    (NONFINITE from the undefined rotation, q stays), above zero nothing."""
    from oracle.inversion import INVERTED, NONFINITE
    g = rng(13)
    X, tets = _mesh(g)
    E = np.zeros((1, 3, 3))
    E[0, 0, 0] = 1.0
    dec = _AffineLatent(E)
    samples = np.array([9, 22, 40])
    q_n = np.array([scale])
    q1, info, _ = fem.fem_step(dec, X, tets, samples, q_n, None, LAM, MU, RHO0, B, 1e-3, GNOptions(max_iter=3))
    assert bool(info.flags & INVERTED) == flag
    if flag:
        assert info.flags & NONFINITE and np.array_equal(q1, q_n)
    _, info, _ = fem.fem_step(dec, X, tets, samples, q_n, None, LAM, MU, RHO0, B, 1e-3, GNOptions(max_iter=3),
                              np.ones(3, np.uint8))
    assert not info.flags & INVERTED
