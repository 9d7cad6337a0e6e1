"""The (m, r, d, width) = (2, 16, 1, 128) decoder: the 2D heat step with a
16-dimensional latent space at width 128 (GPU).

This shape factors its 16 x 16 normal matrix with the row-per-lane
Cholesky, sums 153 partials per batch, and runs its persistent step kernel
with four waves.  Its steps are checked against the FP64 oracle's:

* the linearised step, a single normal-equation solve, on q itself, within
  the Jacobian's normwise error times sqrt(cond(J^T J)) (the least-squares
  perturbation bound);
* both steps on the decoded change at the samples, which the step
  determines, and the Gauss-Newton step on its objective.

The multi-instance Gauss-Newton step beyond 1,024 batches runs as round
kernels; its instances must match their single-instance steps (persistent
kernel) bit for bit."""
import numpy as np
import pytest

from conftest import normwise_rel
from oracle import mlp, step as ostep
from oracle.inversion import GNOptions as OOpts
from workloads import Heat2D

pytestmark = pytest.mark.gpu


def _run(cuda, wl, offsets, y, qn, nu, prec, **opt):
    import torch
    from paper_2206_02607_amd import crom
    dec = crom.Decoder.from_layers(wl.layers, 2, precision=prec, device="cuda:0")
    st = crom.Stepper(dec, offsets, torch.from_numpy(y).to(cuda))
    opt.setdefault("tol_step", 1e-10)
    q1 = st.step(torch.from_numpy(np.atleast_2d(qn)).to(cuda), torch.as_tensor(nu), wl.dt, crom.GNOptions(**opt))
    torch.cuda.synchronize()
    return q1.cpu().numpy(), st.info(), st.targets().cpu().numpy()


def _dg_err(wl, q_gpu, q_ref):
    dec = mlp.MLPDecoder(wl.layers, 2)
    g0 = dec.value(wl.samples, wl.q0)
    return normwise_rel(dec.value(wl.samples, q_gpu) - g0, dec.value(wl.samples, q_ref) - g0)


# Bars on the decoded change and on the latent Jacobian's normwise error
# (the latter times sqrt(cond(J^T J)) bounds the latent update): FP32 as for
# the r = 8 decoder; BF16X3 (split operands on every column) as its low-
# precision test; BF16, whose plain-bfloat16 adjoint leaves the Jacobian
# about 6e-3 off (the decode parity), meets this random network's
# conditioning (sqrt(cond(J^T J)) = 6.4e3 at depth 5): the decoded change is
# reproduced to 0.39 (depth 5, reverse pass) and 0.068 (depth 7, forward
# tangent columns), so its bar only bounds the damage.
TOL = {"fp32": (1e-3, 1e-5), "bf16x3": (2e-3, 1e-4), "bf16": (0.5, 2e-2)}


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "bf16"])
@pytest.mark.parametrize("depth", [5, 7])
def test_step_parity(cuda, prec, depth):
    """Depth 5 forms the latent Jacobian by the reverse pass, depth 7 by
    forward tangent columns; in FP32 and BF16X3 the 20 forward columns at
    width 128 do not fit the LDS, and the library refuses the step.  The
    Gauss-Newton objective after the step is held to the oracle's within 1 %
    (FP32, BF16X3) or 10 % (BF16: measured 3.1 % and 1.5 % above it at
    depths 5 and 7)."""
    from paper_2206_02607_amd import crom
    wl = Heat2D(seed=3, bias_scale=0.1, r=16, depth=depth)
    if prec in ("fp32", "bf16x3") and depth > 6:
        for lin in (True, False):
            with pytest.raises(crom.CromError, match="LDS"):
                _run(cuda, wl, [0, wl.n_samples], wl.samples, wl.q0, [wl.mu], prec, linearized=lin)
        return
    J = mlp.MLPDecoder(wl.layers, 2).value_jac_q(wl.samples, wl.q0)[1].reshape(-1, wl.r)
    sq = np.sqrt(np.linalg.cond(J.T @ J))
    tol_dg, tol_j = TOL[prec]
    for lin in (True, False):
        q1, info, f = _run(cuda, wl, [0, wl.n_samples], wl.samples, wl.q0, [wl.mu], prec, linearized=lin)
        qr, oinfo, fr = ostep.heat_step(mlp.MLPDecoder(wl.layers, 2), wl.samples, wl.q0, wl.mu, wl.dt,
                                        OOpts(max_iter=5, linearized=lin, tol_step=1e-12))
        e_f = normwise_rel(f, fr)
        e_dg = _dg_err(wl, q1[0], qr)
        e_q = normwise_rel(q1[0] - wl.q0, qr - wl.q0)
        print(f"r16 depth {depth} {prec} lin={lin}: targets {e_f:.2e} dg {e_dg:.2e} dq {e_q:.2e} "
              f"sqrt cond {sq:.2e} flags {info['flags'][0]} iters {info['iters'][0]}/{oinfo.iters} "
              f"obj {info['obj_last'][0]:.4e}/{oinfo.obj_last:.4e}")
        assert e_f <= (1e-5 if prec == "fp32" else 1e-4)
        assert e_dg <= tol_dg
        if lin:
            assert e_q <= tol_j * sq
        else:
            rel = 1.1 if prec == "bf16" else 1.01
            assert info["obj_last"][0] <= oinfo.obj_last * rel + 1e-3 * oinfo.obj_first


def test_batched_rounds_equal_single(cuda):
    """Nine instances of 2,000 samples (1,125 batches: the round kernels)
    reproduce the persistent kernel's single-instance steps bit for bit
    (iterates, flags, iterations, trials and objectives; only the round
    count may differ, as for the r = 8 decoder)."""
    wl = Heat2D(seed=4, bias_scale=0.1, r=16)
    g = np.random.Generator(np.random.PCG64(11))
    n = 9
    qn = wl.q0[None] + 0.1 * g.uniform(-1, 1, size=(n, wl.r))
    nu = 0.1 + 0.9 * g.uniform(size=n)
    y = np.tile(wl.samples, (n, 1))
    offsets = np.arange(n + 1, dtype=np.int64) * wl.n_samples
    qb, ib, _ = _run(cuda, wl, offsets, y, qn, nu, "bf16", max_iter=5)
    print(f"iterations {ib['iters'].tolist()} trials {ib['ls_evals'].tolist()} flags {ib['flags'].tolist()}")
    for i in (0, 4, 8):
        q1, i1, _ = _run(cuda, wl, [0, wl.n_samples], wl.samples, qn[i], [nu[i]], "bf16", max_iter=5)
        np.testing.assert_array_equal(qb[i], q1[0])
        for k in ("flags", "iters", "ls_evals", "obj_first", "obj_last"):
            assert ib[i][k] == i1[0][k], k
        assert ib[i]["rounds"] >= i1[0]["rounds"]  # objective-only rounds after rejected trials
