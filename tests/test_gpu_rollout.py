"""2D heat end to end on the GPU (GPU): FP64 finite-difference snapshots,
decoder and encoder trained by the library's own kernels, latent rollouts
judged by the FP64 finite-difference solution.

* Gain of training: the trained network's rollout error (space-time relative
  L2 over the recorded states) is a few percent, the untrained network's
  (same architecture, same initial weights, no training) is about 100%.
* Precision: rollouts of the same trained network with the FP32 and the
  BF16 decoder arithmetic reach the same error (the rollout error is the
  network's approximation error, far above either arithmetic's).
The training is 20,000 Adam steps (about 30 s).  Shorter runs are fragile:
a low reconstruction loss does not by itself give the network an accurate
Laplacian, and at 8,000 steps the rollout error ranged from 4 % to 57 %
over three batch orders; at 20,000 steps it was 2.7-5.2 %."""
import numpy as np
import pytest

from workloads import Train2D

pytestmark = pytest.mark.gpu

TRAIN_STEPS = 20000


@pytest.fixture(scope="module")
def trained(cuda):
    import torch
    from paper_2206_02607_amd import crom, heat2d
    w = Train2D()
    u0 = w.initial_field()
    snaps = heat2d.fd_snapshots(u0, w.mu, w.times, w.dx, w.dt_fd, cuda)
    rows = snaps.reshape(-1, w.grid * w.grid)
    nodes = torch.from_numpy(w.nodes).to(cuda)
    sd = heat2d.Standardization.of(rows, nodes)
    enc0 = np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in w.enc_layers]).astype(np.float32)
    nets = {}
    for name, steps in (("trained", TRAIN_STEPS), ("untrained", 0)):
        dec = crom.Decoder.from_layers(w.layers, w.m, precision="bf16", device=cuda)
        T = crom.Trainer(dec, enc0.copy(), w.enc_hidden, sd.points(nodes), w.batch)
        losses = heat2d.train(T, sd.data(rows), steps, seed=1) if steps else None
        sd.fold(dec, T.enc_params, T.n_in, T.hidden)
        q0 = T.encode(torch.from_numpy(u0.astype(np.float32)).to(cuda).reshape(1, -1))
        nets[name] = (dec, q0.cpu().numpy().astype(np.float64), losses)
        if name == "trained":
            nets["enc"] = (T.enc_params.detach().clone(), T.hidden)
    mus = np.concatenate([w.mu_test, w.mu[:2]])
    record = [0, 125, 250, 375, 500]
    ref = heat2d.fd_snapshots(u0, mus, [k * w.dt for k in record], w.dx, w.dt_fd, cuda)
    refs = [ref[:, k].reshape(len(mus), -1) for k in range(len(record))]
    return w, nodes, nets, mus, record, refs, rows


BROKEN = 2 | 4 | 16  # SINGULAR, NONFINITE, ABORTED


def _rollout_error(w, nodes, dec, q0, mus, record, refs, linearized):
    """Space-time rollout error per instance.  The flags of every step are
    collected: no step may end SINGULAR, NONFINITE or ABORTED; a
    Gauss-Newton step that ends LS_FAIL (no further decrease resolvable at
    the step tolerance) keeps its last accepted iterate and is reported."""
    from paper_2206_02607_amd import crom, heat2d
    opts = crom.GNOptions(max_iter=5, linearized=linearized, tol_step=1e-6)
    ro = heat2d.rollout(dec, np.tile(q0, (len(mus), 1)), w.nodes[w.sample_idx], mus, w.dt, record[-1], opts,
                        record)
    assert np.all(ro.flags[-1] & BROKEN == 0), ro.flags[-1]
    if linearized:
        assert np.all(ro.flags[-1] & crom.FLAG_LS_FAIL == 0)
    print("flags over the rollout (OR per instance)", ro.flags[-1].tolist())
    fields = [heat2d.decode_fields(dec, nodes, q) for q in ro.q]
    return heat2d.spacetime_error(fields, refs), ro


def _untrained_error(w, nodes, dec, q0, mus, record, refs, linearized):
    """The untrained network's rollout (its steps may fail: it is not a
    model of the field)."""
    from paper_2206_02607_amd import crom, heat2d
    opts = crom.GNOptions(max_iter=5, linearized=linearized, tol_step=1e-6)
    ro = heat2d.rollout(dec, np.tile(q0, (len(mus), 1)), w.nodes[w.sample_idx], mus, w.dt, record[-1], opts,
                        record)
    fields = [heat2d.decode_fields(dec, nodes, q) for q in ro.q]
    return heat2d.spacetime_error(fields, refs), ro


def test_training_converges(trained):
    _, _, nets, _, _, _, _ = trained
    losses = nets["trained"][2]
    print("loss", losses[:50].mean(), losses[-50:].mean())
    assert losses[-200:].mean() < 2e-3 * losses[:50].mean()


def test_initial_field_reconstruction(trained):
    """Decoding the encoder's latent of the initial field reproduces it to a
    few percent (the encoder and decoder are used in physical units, after
    the standardization was folded into their weights)."""
    from paper_2206_02607_amd import heat2d
    w, nodes, nets, _, _, _, rows = trained
    dec, q0, _ = nets["trained"]
    err = heat2d.rel_error(heat2d.decode_fields(dec, nodes, q0), rows[0:1])[0]
    print("initial-field reconstruction", err)
    assert err < 0.05


@pytest.mark.parametrize("linearized", [0, 1])
def test_trained_vs_untrained_rollout(trained, linearized):
    w, nodes, nets, mus, record, refs, _ = trained
    e_t, ro_t = _rollout_error(w, nodes, nets["trained"][0], nets["trained"][1], mus, record, refs, linearized)
    e_u, _ = _untrained_error(w, nodes, nets["untrained"][0], nets["untrained"][1], mus, record, refs, linearized)
    print("space-time rollout error: trained", e_t.round(4), "untrained", e_u.round(3), "GN iters", ro_t.iters)
    assert np.all(np.isfinite(e_t))
    assert e_t.max() < 0.08
    assert e_u.min() > 0.5
    assert e_t.max() < 0.1 * e_u.min()


def test_bf16_and_fp32_reach_equal_rollout_error(trained):
    from paper_2206_02607_amd import crom
    w, nodes, nets, mus, record, refs, _ = trained
    dec, q0, _ = nets["trained"]
    errs = {}
    for prec in ("fp32", "bf16"):
        d = crom.Decoder(dec.params.detach().clone(), dec.m, dec.r, dec.d, dec.width, dec.depth, prec, nodes.device)
        errs[prec], _ = _rollout_error(w, nodes, d, q0, mus, record, refs, 1)
    print("LLS rollout error fp32", errs["fp32"].round(5), "bf16", errs["bf16"].round(5))
    assert np.abs(errs["fp32"] - errs["bf16"]).max() < 0.1 * errs["fp32"].min()


def test_robust_sampling_beats_random_sets(trained):
    """Appendix "Robust Sampling": greedy selection from 12 random interior
    nodes to 24 (10 candidates per round, the final-time residual summed
    over 10 training diffusivities) ends with a lower metric (mean + max of
    the residual vector) than each of four random interior sets of 24
    nodes."""
    import torch
    from paper_2206_02607_amd import crom
    w, nodes, nets, _, _, _, rows = trained
    dec, q0, _ = nets["trained"]
    ks = np.arange(0, w.n_mu, 4)
    n_mu = len(ks)
    nt = len(w.times)
    ref = rows.reshape(w.n_mu, nt, -1)[ks, nt - 1].to(torch.float64).reshape(n_mu, -1, 1).contiguous()
    n_steps = int(round(w.times[-1] / w.dt))
    gi = np.arange(w.grid)
    edge = (gi == 0) | (gi == w.grid - 1)
    clamp = (edge[:, None] | edge[None, :]).reshape(-1).astype(np.uint8)
    interior = np.flatnonzero(clamp == 0)
    g = np.random.Generator(np.random.PCG64(21))
    opts = crom.GNOptions(max_iter=1, linearized=True)
    args = (dec, nodes, ref, np.tile(q0, (n_mu, 1)), w.mu[ks], w.dt)
    kw = dict(opts=opts, node_clamp=torch.from_numpy(clamp).to(nodes.device))
    greedy = crom.robust_sampling(*args, g.choice(interior, 12, replace=False), n_steps, target=0.0, n_try=10,
                                  max_samples=24, **kw)
    rand = [crom.robust_sampling(*args, g.choice(interior, 24, replace=False), n_steps, target=0.0,
                                 max_samples=24, **kw).metric for _ in range(4)]
    print("greedy metric", greedy.metric, "samples", greedy.samples.tolist(), "random sets", np.round(rand, 4))
    assert greedy.rounds == 12
    assert greedy.metric < min(rand)


def test_trained_crom_vs_pod(trained):
    """The learned decoder against the linear baseline the paper compares
    with (Sec. "Comparison with Prior Approaches"): POD with the same latent
    dimension r = 8, its basis the leading singular vectors of the same 200
    FP64 training snapshots (the finite-difference solver's, bit-exact with
    the oracle's solver), stepped by the method's own heat update (its
    Laplacian the full-order stencil applied to the basis) and linearised
    inversion at the same 500 sample nodes, from the projection of the
    initial field.  Both rollouts are judged by the FP64 finite-difference
    solution over 500 steps for the held-out and two training diffusivities;
    both errors are printed, with the memory each needs for its manifold."""
    from oracle import pod, step as ostep
    from oracle.inversion import GNOptions
    w, nodes, nets, mus, record, refs, rows = trained
    dec, q0, _ = nets["trained"]
    e_crom, _ = _rollout_error(w, nodes, dec, q0, mus, record, refs, 1)
    U = pod.pod_basis(rows.cpu().numpy(), w.r)
    P = pod.PODDecoder(U, w.grid, w.grid, w.dx)
    u0 = w.initial_field().ravel()
    opts = GNOptions(max_iter=1, linearized=True)
    e_pod = []
    for k, mu in enumerate(mus):
        q = P.encode(u0)
        num = den = 0.0
        for n in range(record[-1] + 1):
            if n in record:
                ref = refs[record.index(n)][k].cpu().numpy()
                num += float(((P.decode(q) - ref) ** 2).sum())
                den += float((ref ** 2).sum())
            if n < record[-1]:
                q, info, _ = ostep.heat_step(P, w.sample_idx, q, float(mu), w.dt, opts)
                assert info.flags == 0
        e_pod.append(np.sqrt(num / den))
    e_pod = np.array(e_pod)
    mem_crom, mem_pod = dec.params.numel(), U.size
    print("space-time rollout error, r = 8: CROM", e_crom.round(4), "POD", e_pod.round(4),
          f"| manifold parameters: CROM {mem_crom}, POD {mem_pod} ({mem_pod / mem_crom:.2f}x)")
    assert np.all(np.isfinite(e_pod)) and np.all(e_pod < 1.0)
    # the network's size does not grow with the discretisation: at this grid
    # it already needs about half the values of the r = 8 basis
    assert mem_crom < 0.6 * mem_pod


def test_fd_fallback_carries_a_failed_instance(trained):
    """An instance whose samples all sit on one node has a rank-one J^T J:
    every step ends SINGULAR and keeps q_n, so alone its field never
    changes.  With the full-order fallback (crom_heat_fallback: decode at
    every node, FP64 finite-difference update over the step, projection back
    onto the decoder at every node) the rollout continues from the
    full-order update; the judged error is then close to the healthy
    instances', while without the fallback it is that of a frozen field.  The healthy instances of the batch are bit-identical
    with and without the fallback."""
    import torch
    from paper_2206_02607_amd import crom, heat2d
    w, nodes, nets, mus, record, refs, _ = trained
    dec, q0, _ = nets["trained"]
    S = len(w.sample_idx)
    y = np.tile(w.nodes[w.sample_idx], (len(mus), 1)).astype(np.float32)
    bad = 1
    y[bad * S:(bad + 1) * S] = w.nodes[w.sample_idx[S // 2]]
    offsets = np.arange(len(mus) + 1, dtype=np.int64) * S
    opts = crom.GNOptions(max_iter=1, linearized=True)
    fb = crom.HeatFallback(dec, nodes, w.grid, w.grid, w.dx, w.dt_fd)
    runs = {}
    for name, f in (("plain", None), ("fallback", fb)):
        ro = heat2d.rollout(dec, np.tile(q0, (len(mus), 1)), y, mus, w.dt, record[-1], opts, record,
                            offsets=offsets, fallback=f)
        fields = [heat2d.decode_fields(dec, nodes, q) for q in ro.q]
        runs[name] = (heat2d.spacetime_error(fields, refs), ro)
    e_plain, ro_plain = runs["plain"]
    e_fb, ro_fb = runs["fallback"]
    print("rollout error without fallback", e_plain.round(4), "with", e_fb.round(4),
          "fallback steps", ro_fb.fallbacks.tolist())
    assert ro_plain.flags[-1][bad] & crom.FLAG_SINGULAR
    assert ro_fb.fallbacks[bad] == record[-1]
    good = [k for k in range(len(mus)) if k != bad]
    assert np.all(ro_fb.fallbacks[good] == 0)
    for qa, qb in zip(ro_plain.q, ro_fb.q):
        assert np.array_equal(qa[good], qb[good])
    # frozen without the fallback; tracked with it
    assert np.array_equal(ro_plain.q[-1][bad], q0[0])
    assert e_fb[bad] < 0.1 and e_fb[bad] < 0.25 * e_plain[bad]
