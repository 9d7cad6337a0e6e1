"""Parity of the corotated finite-element latent step (crom_step with
CROM_PDE_COROTATED_FE) with the FP64 oracle (GPU).

The decoder is the elastic bar's, (X in R^3, q in R^16) -> 6 x ELU width
256 -> 3, output scaled by 1e-2; the mesh is a jittered box of linear
tetrahedra (six per cube); lam = 2.5e4, mu = 6.5e4, rho0 = 1000, gravity.

* The ring decode (the displacement at every vertex of the samples' one-ring)
  against the oracle's decoder: FP32 1e-5, BF16 1e-4 normwise (the value
  column's bars).
* The finite-element kernel alone: the oracle's update computed from the
  GPU's own ring displacements (substituted through a lookup decoder) must
  match the GPU's increments to 1e-9 normwise; both sides are FP64 from the
  same FP32 inputs and differ only in the order of sums and in how the
  rotation is found (Newton's iteration here, the SVD in the oracle).  At
  the bar's full size (64 x 16 x 16 vertices, 500 samples) on every sample.
* The velocity term (q_prev given) through the FP32/BF16 latent Jacobian:
  its error relative to the velocity part itself within the derivative
  bars, FP32 1e-5 and BF16 2e-2.
* The Gauss-Newton latent update against the oracle's step, within ten
  times the condition number of J times the measured relative error of the
  increments (the targets' error passes to the least-squares solution
  amplified by at most cond(J)).
* A batch of instances reproduces each instance run alone bit for bit, and
  corrupted stencil data makes only its own instance NONFINITE."""
import numpy as np
import pytest

from conftest import normwise_rel
from oracle import fem, mlp
from oracle.inversion import GNOptions
from workloads import Corotated3D, box_tet_mesh, rng

pytestmark = pytest.mark.gpu

LAM, MU, RHO0 = 2.5e4, 6.5e4, 1000.0
GRAV = (0.0, 0.0, -9.81)
DT = 1e-3
TOL_VALUE = {"fp32": 1e-5, "bf16": 1e-4}
TOL_DERIV = {"fp32": 1e-5, "bf16": 2e-2}


def _coef(mu=MU, lam=LAM, B=GRAV):
    return np.array([lam, mu, RHO0, *B], dtype=np.float64)


@pytest.fixture(scope="module")
def small():
    w = Corotated3D(n_samples=1)  # decoder only
    g = rng(41)
    X, tets = box_tet_mesh(10, 5, 5, 1.0 / 15.0, 0.15, g)
    samples = np.sort(g.choice(X.shape[0], size=40, replace=False))
    q0 = g.uniform(-0.1, 0.1, size=w.r)
    return w.layers, X, tets, samples, q0


class _Lookup:
    """Decoder stand-in returning the GPU's ring displacements (found by
    position) and, when given, the oracle decoder's latent Jacobian."""

    def __init__(self, X, ring_vert, ring_u, odec=None):
        self.u = {tuple(X[v].astype(np.float64)): ring_u[i] for i, v in enumerate(ring_vert)}
        self.odec, self.r = odec, 16

    def value(self, Y, q):
        return np.stack([self.u[tuple(y)] for y in np.asarray(Y, dtype=np.float64)]).astype(np.float64)

    def value_jac_q(self, Y, q):
        J = self.odec.value_jac_q(Y, q)[1] if self.odec else np.zeros((len(Y), 3, self.r))
        return self.value(Y, q), J


def _run(crom, dec, X, tets, samples, coef, q_n, q_prev, opts, cuda, stencil=None):
    """One step over the instances `samples` (a list of vertex arrays);
    returns (q_next, info, increments, ring_u, stencil)."""
    import torch
    st_mesh = stencil or crom.FEStencil(X, tets, samples, cuda)
    st = crom.Stepper(dec, st_mesh.offsets, st_mesh.y, pde="corotated_fe", mesh=st_mesh)
    qn = torch.from_numpy(np.atleast_2d(q_n)).to(cuda)
    qp = None if q_prev is None else torch.from_numpy(np.atleast_2d(q_prev)).to(cuda)
    q1 = st.step(qn, torch.from_numpy(np.atleast_2d(coef)).to(cuda), DT, opts, q_prev=qp)
    torch.cuda.synchronize()
    return (q1.cpu().numpy(), st.info(), st.increments().cpu().numpy(),
            st_mesh.ring_u[:st_mesh.n_ring].cpu().numpy(), st_mesh)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_ring_decode_and_fe_kernel(cuda, small, prec):
    from paper_2206_02607_amd import crom
    layers, X, tets, samples, q0 = small
    dec = crom.Decoder.from_layers(layers, 3, precision=prec, device=cuda)
    _, info, inc, ring_u, sm = _run(crom, dec, X, tets, [samples], _coef(), q0, None,
                                    crom.GNOptions(max_iter=1, linearized=True), cuda)
    assert info["flags"][0] == 0
    odec = mlp.MLPDecoder(layers, 3)
    ref_u = odec.value(X[sm.ring_vert].astype(np.float64), q0)
    err_u = normwise_rel(ring_u, ref_u)
    _, ref_inc = fem.fem_targets(_Lookup(X, sm.ring_vert, ring_u), X, tets, samples, q0, None, LAM, MU, RHO0,
                                 GRAV, DT)
    err_k = normwise_rel(inc, ref_inc)
    _, full = fem.fem_targets(odec, X, tets, samples, q0, None, LAM, MU, RHO0, GRAV, DT)
    print(f"{prec}: ring {sm.n_ring} vertices, decode error {err_u:.2e}; FE kernel vs oracle on the GPU's "
          f"ring values {err_k:.2e}; increments vs the full oracle {normwise_rel(inc, full):.2e} "
          f"(|inc| {np.abs(full).max():.2e}, gravity part {DT * DT * 9.81:.1e})")
    assert err_u <= TOL_VALUE[prec]
    assert err_k <= 1e-9


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_velocity_term(cuda, small, prec):
    from paper_2206_02607_amd import crom
    layers, X, tets, samples, q0 = small
    dec = crom.Decoder.from_layers(layers, 3, precision=prec, device=cuda)
    q_prev = q0 - 0.01 * rng(42).uniform(-1, 1, size=q0.size)
    _, info, inc, ring_u, sm = _run(crom, dec, X, tets, [samples], _coef(), q0, q_prev,
                                    crom.GNOptions(max_iter=1, linearized=True), cuda)
    odec = mlp.MLPDecoder(layers, 3)
    look = _Lookup(X, sm.ring_vert, ring_u, odec)
    _, with_v = fem.fem_targets(look, X, tets, samples, q0, q_prev, LAM, MU, RHO0, GRAV, DT)
    _, without_v = fem.fem_targets(look, X, tets, samples, q0, None, LAM, MU, RHO0, GRAV, DT)
    v_part = with_v - without_v
    err = np.linalg.norm(inc - with_v) / np.linalg.norm(v_part)
    print(f"{prec}: |dt v| {np.abs(v_part).max():.2e}, error relative to it {err:.2e}")
    assert err <= TOL_DERIV[prec]


def _cond(layers, X, q):
    J = mlp.decode_jets(layers, X.astype(np.float64), q, 3)[3].reshape(-1, q.size)
    s = np.linalg.svd(J, compute_uv=False)
    return s[0] / s[-1]


@pytest.mark.parametrize("linearized", [1, 0])
def test_step_parity_fp32(cuda, small, linearized):
    from paper_2206_02607_amd import crom
    layers, X, tets, samples, q0 = small
    dec = crom.Decoder.from_layers(layers, 3, precision="fp32", device=cuda)
    q_prev = q0 - 0.01 * rng(43).uniform(-1, 1, size=q0.size)
    opts = dict(max_iter=5, linearized=bool(linearized), tol_step=1e-10)
    q1, info, inc, _, _ = _run(crom, dec, X, tets, [samples], _coef(), q0, q_prev, crom.GNOptions(**opts), cuda)
    odec = mlp.MLPDecoder(layers, 3)
    ref, rinfo, _ = fem.fem_step(odec, X, tets, samples, q0, q_prev, LAM, MU, RHO0, GRAV, DT, GNOptions(**opts))
    _, ref_inc = fem.fem_targets(odec, X, tets, samples, q0, q_prev, LAM, MU, RHO0, GRAV, DT)
    e_inc = normwise_rel(inc, ref_inc)
    kappa = _cond(layers, X[samples], q0)
    err = normwise_rel(q1[0] - q0, ref - q0)
    bound = 10.0 * kappa * max(e_inc, 1e-7)
    print(f"linearized={linearized}: |dq| {np.abs(ref - q0).max():.3e} error {err:.2e} (increments {e_inc:.2e}, "
          f"cond(J) {kappa:.1f}, bound {bound:.2e}) flags {info['flags'][0]} iters {info['iters'][0]} "
          f"(oracle {rinfo.flags} {rinfo.iters})")
    assert err <= bound
    assert info["flags"][0] & ~crom.FLAG_MAXITER == 0


def test_batched_equals_single(cuda, small):
    from paper_2206_02607_amd import crom
    layers, X, tets, _, q0 = small
    dec = crom.Decoder.from_layers(layers, 3, precision="bf16", device=cuda)
    g = rng(44)
    n = 3
    sets = [np.sort(g.choice(X.shape[0], size=s, replace=False)) for s in (23, 40, 17)]
    qn = q0[None] + 0.05 * g.uniform(-1, 1, size=(n, q0.size))
    qp = qn - 0.01 * g.uniform(-1, 1, size=(n, q0.size))
    coef = np.stack([_coef(mu=6e4 + 5e3 * i) for i in range(n)])
    opts = crom.GNOptions(max_iter=5, tol_step=1e-8)
    qb, ib, incb, _, sm = _run(crom, dec, X, tets, sets, coef, qn, qp, opts, cuda)
    off = sm.offsets.cpu().numpy()
    for i in range(n):
        q1, i1, inc1, _, _ = _run(crom, dec, X, tets, [sets[i]], coef[i], qn[i], qp[i], opts, cuda)
        np.testing.assert_array_equal(qb[i], q1[0])
        np.testing.assert_array_equal(incb[off[i]:off[i + 1]], inc1)
        assert ib[i].tobytes() == i1[0].tobytes()


def test_corrupt_stencil_is_contained(cuda, small):
    """A corner outside 0..3 in instance 0 and a ring index past the ring in
    instance 1 make those instances NONFINITE; instance 2 is untouched."""
    from paper_2206_02607_amd import crom
    layers, X, tets, samples, q0 = small
    dec = crom.Decoder.from_layers(layers, 3, precision="fp32", device=cuda)
    sets = [samples[:10], samples[10:25], samples[25:]]
    sm = crom.FEStencil(X, tets, sets, cuda)
    inc_off = sm.inc_offsets.cpu().numpy()
    sm.inc_corner[int(inc_off[3])] = 9
    sm.inc_tets[int(inc_off[12]), 2] = 1 << 20
    q = np.tile(q0, (3, 1))
    opts = crom.GNOptions(max_iter=2)
    _, info, _, _, _ = _run(crom, dec, X, tets, sets, np.tile(_coef(), (3, 1)), q, None, opts, cuda, stencil=sm)
    print("flags", info["flags"])
    assert info["flags"][0] & crom.FLAG_NONFINITE
    assert info["flags"][1] & crom.FLAG_NONFINITE
    assert info["flags"][2] & ~crom.FLAG_MAXITER == 0


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_full_size_fe_kernel(cuda, prec):
    """The bar of 64 x 16 x 16 vertices with 500 samples, as timed: the FE
    kernel against the oracle on the GPU's own ring values, every sample.
    The step itself ends without a failure; the line search may find no
    decrease the arithmetic resolves before the iteration cap (LS_FAIL at
    iteration 3 in both arithmetics: where depends on the low bits of the
    sums), a valid end as in the batched heat test."""
    from paper_2206_02607_amd import crom
    w = Corotated3D()
    dec = crom.Decoder.from_layers(w.layers, 3, precision=prec, device=cuda)
    coef = _coef(mu=w.mu[0], lam=w.lam)
    _, info, inc, ring_u, sm = _run(crom, dec, w.X, w.tets, w.samples, coef, w.q0[0], None,
                                    crom.GNOptions(max_iter=5), cuda)
    _, ref = fem.fem_targets(_Lookup(w.X, sm.ring_vert, ring_u), w.X, w.tets, w.samples[0], w.q0[0], None,
                             w.lam, w.mu[0], w.rho0, w.gravity, w.dt)
    err = normwise_rel(inc, ref)
    print(f"{prec}: ring {sm.n_ring} vertices, {sm.n_inc} incidences; FE kernel error {err:.2e}; "
          f"flags {info['flags'][0]} iters {info['iters'][0]}")
    assert err <= 1e-9
    assert info["flags"][0] & ~(crom.FLAG_MAXITER | crom.FLAG_LS_FAIL) == 0


def test_full_size_batched_fe_kernel(cuda):
    """Two instances of the bar (500 samples each, different sample sets and
    shear moduli) in one step: each instance's increments against the
    oracle on the GPU's own ring values."""
    from paper_2206_02607_amd import crom
    w = Corotated3D(n_inst=2, seed=3)
    dec = crom.Decoder.from_layers(w.layers, 3, precision="bf16", device=cuda)
    coef = np.stack([_coef(mu=w.mu[i], lam=w.lam) for i in range(2)])
    _, info, inc, ring_u, sm = _run(crom, dec, w.X, w.tets, w.samples, coef, w.q0, None,
                                    crom.GNOptions(max_iter=1, linearized=True), cuda)
    roff = sm.ring_offsets.cpu().numpy()
    off = sm.offsets.cpu().numpy()
    for i in range(2):
        a, b = roff[i], roff[i + 1]
        look = _Lookup(w.X, sm.ring_vert[a:b], ring_u[a:b])
        _, ref = fem.fem_targets(look, w.X, w.tets, w.samples[i], w.q0[i], None, w.lam, w.mu[i], w.rho0,
                                 w.gravity, w.dt)
        err = normwise_rel(inc[off[i]:off[i + 1]], ref)
        print(f"instance {i}: ring {b - a} vertices, FE kernel error {err:.2e}, flags {info['flags'][i]}")
        assert err <= 1e-9
        assert info["flags"][i] == 0


def test_instance_without_samples(cuda, small):
    """A batch whose middle instance has no samples: that instance ends at
    once as SINGULAR with q_{n+1} = q_n, the others match their runs alone."""
    from paper_2206_02607_amd import crom
    layers, X, tets, samples, q0 = small
    dec = crom.Decoder.from_layers(layers, 3, precision="fp32", device=cuda)
    sets = [samples[:20], np.zeros(0, dtype=np.int64), samples[20:]]
    g = rng(45)
    qn = q0[None] + 0.02 * g.uniform(-1, 1, size=(3, q0.size))
    coef = np.tile(_coef(), (3, 1))
    opts = crom.GNOptions(max_iter=3, tol_step=1e-8)
    qb, ib, incb, _, sm = _run(crom, dec, X, tets, sets, coef, qn, None, opts, cuda)
    assert ib["flags"][1] == crom.FLAG_SINGULAR
    np.testing.assert_array_equal(qb[1], qn[1])
    for i in (0, 2):
        q1, i1, _, _, _ = _run(crom, dec, X, tets, [sets[i]], coef[i], qn[i], None, opts, cuda)
        np.testing.assert_array_equal(qb[i], q1[0])
        assert ib[i].tobytes() == i1[0].tobytes()


def test_initial_guess_in_fe_step(cuda, small):
    """crom_step_guess on the FE step (the elastic persistent kernel): a
    worse guess leaves the step bit-identical to crom_step (one more round);
    the converged latent of a long run as the guess ends one iteration at
    an objective no higher than three iterations from q_n reach."""
    import torch
    from paper_2206_02607_amd import crom
    layers, X, tets, samples, q0 = small
    dec = crom.Decoder.from_layers(layers, 3, precision="fp32", device=cuda)
    sm = crom.FEStencil(X, tets, [samples], cuda)
    st = crom.Stepper(dec, sm.offsets, sm.y, pde="corotated_fe", mesh=sm)
    coef = torch.from_numpy(_coef()[None]).to(cuda)
    qn = torch.from_numpy(q0[None]).to(cuda)
    q_long = st.step(qn, coef, DT, crom.GNOptions(max_iter=20, tol_step=1e-12)).clone()
    obj_long = st.info()["obj_last"][0]
    q3 = st.step(qn, coef, DT, crom.GNOptions(max_iter=3, tol_step=1e-12)).cpu().numpy()
    i3 = st.info()[0]
    q_bad = st.step(qn, coef, DT, crom.GNOptions(max_iter=3, tol_step=1e-12), q_init=qn + 0.5).cpu().numpy()
    ib = st.info()[0]
    np.testing.assert_array_equal(q_bad, q3)
    for k in ("flags", "iters", "ls_evals", "obj_first", "obj_last"):
        assert ib[k] == i3[k], k
    assert ib["rounds"] == i3["rounds"] + 1
    st.step(qn, coef, DT, crom.GNOptions(max_iter=1, tol_step=1e-12), q_init=q_long)
    ig = st.info()[0]
    print(f"objective: q_n {i3['obj_first']:.4e}, 3 iterations {i3['obj_last']:.4e}, long run {obj_long:.4e}, "
          f"1 iteration from the guess {ig['obj_last']:.4e}")
    assert ig["obj_first"] == i3["obj_first"]
    assert ig["obj_last"] <= i3["obj_last"] * (1 + 1e-9)


@pytest.mark.parametrize("scale", [1.0, -1000.0])
def test_inverted_flag(cuda, small, scale):
    """The decoder's output layer scaled by `scale`: the oracle's rule (a
    tetrahedron incident on a free sample with det F <= 0) decides whether
    the step reports INVERTED; the GPU agrees, and an inverted instance also
    reports NONFINITE and keeps q_n."""
    from paper_2206_02607_amd import crom
    from oracle.inversion import INVERTED
    layers, X, tets, samples, q0 = small
    layers = [(np.asarray(W, np.float64), np.asarray(b, np.float64)) for W, b in layers]
    layers[-1] = (layers[-1][0] * scale, layers[-1][1] * scale)
    odec = mlp.MLPDecoder(layers, 3)
    expect = fem.inverted(odec, X, tets, samples, q0)
    # the sign of det F must not hinge on rounding: every incident det F of
    # a free sample is either clearly positive, or one is clearly negative
    inc, ring = fem.one_ring(tets, samples)
    x = np.full_like(X, np.nan, dtype=np.float64)
    x[ring] = X[ring] + odec.value(X[ring].astype(np.float64), q0)
    dets = np.array([np.linalg.det(fem.deformation_gradient(x, X, tets[t])) for ts in inc for t in ts])
    assert (dets.min() < -0.05) if expect else (dets.min() > 0.05)
    dec = crom.Decoder.from_layers(layers, 3, precision="fp32", device=cuda)
    q1, info, _, _, _ = _run(crom, dec, X, tets, [samples], _coef(), q0, None,
                             crom.GNOptions(max_iter=3, tol_step=1e-6), cuda)
    print(f"scale {scale}: min det F {dets.min():.3f}, flags {info['flags'][0]}, oracle inverted {expect}")
    assert bool(info["flags"][0] & crom.FLAG_INVERTED) == expect
    assert crom.FLAG_INVERTED == INVERTED
    if expect:
        assert info["flags"][0] & crom.FLAG_NONFINITE
        assert np.array_equal(q1[0], q0)
