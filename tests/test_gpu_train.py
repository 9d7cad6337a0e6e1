"""Parity of the hand-written training kernels (crom_train_grads,
crom_adam_step, crom_train_step, crom_decode_vjp and the autograd wrapper)
with the FP64 training oracle (GPU).

Tolerances, normwise relative per tensor: 1e-5 in FP32 and 2e-2 in the
bfloat16 modes (bfloat16 keeps 8 significant bits, 2^-9 relative rounding per
stored activation and operand, accumulated over a handful of layers and
averaged over hundreds of rows).  The bfloat16 path differentiates the
network whose matrix-core weights (decoder hidden-to-hidden layers, the
encoder's first layer) are held in bfloat16, as mixed-precision training
does; its reference is the oracle at those rounded weights.  Rounding the
weights is a perturbation of the model, not an error of the derivative: on
random targets, where the residual sums behind the bias gradients cancel,
it moves them by up to 4e-2 (printed as `vs_fp32_weights`).
The sizes are ragged on purpose: rows of the decoder batch, the encoder's
input and hidden widths are not multiples of the 64 x 64 matrix tile, and
the weight-gradient products take the split-K path with a short last
chunk."""
import numpy as np
import pytest

from conftest import normwise_rel
from oracle import train
from workloads import rng, uniform_points, xavier_mlp

pytestmark = pytest.mark.gpu

SHAPES = {"1d": (1, 3, 1, 32, 5), "2d": (2, 8, 1, 128, 5), "3d": (3, 16, 3, 256, 6)}
TOL = {"fp32": 1e-5, "bf16": 2e-2}


def _problem(shape, seed, B, P, hidden=40):
    m, r, d, w, depth = SHAPES[shape]
    g = rng(seed)
    dec = xavier_mlp(g, m, r, d, w, depth, bias_scale=0.2)
    enc = xavier_mlp(g, P * d, 0, r, hidden, 1, bias_scale=0.2)
    x = uniform_points(g, P, m)
    u = g.uniform(-1, 1, size=(B, P * d)).astype(np.float32)
    return dec, enc, x, u, m


def _flat(layers):
    return np.concatenate([np.concatenate([np.asarray(W, np.float32).ravel(), np.asarray(b, np.float32).ravel()])
                           for W, b in layers])


def _split(flat, layers):
    out, off = [], 0
    for W, b in layers:
        nW, nb = W.size, b.size
        out.append((flat[off:off + nW].reshape(W.shape), flat[off + nW:off + nW + nb]))
        off += nW + nb
    return out


def _bf16(a):
    """Round to the nearest bfloat16 (ties to even), on the CPU."""
    import torch
    return torch.from_numpy(np.asarray(a, np.float32)).to(torch.bfloat16).to(torch.float32).numpy()


def _as_held(dec, enc, prec):
    """The parameters as the GPU path holds them: FP32, and in the bfloat16
    modes the matrix-core weights rounded to bfloat16."""
    d32 = [(np.asarray(W, np.float32), np.asarray(b, np.float32)) for W, b in dec]
    e32 = [(np.asarray(W, np.float32), np.asarray(b, np.float32)) for W, b in enc] if enc else None
    if prec == "fp32":
        return d32, e32
    d32 = [d32[0]] + [(_bf16(W), b) for W, b in d32[1:-1]] + [d32[-1]]
    if e32:
        e32 = [(_bf16(e32[0][0]), e32[0][1])] + e32[1:]
    return d32, e32


def _trainer(dec, enc, x, u, m, prec, cuda, hidden=40):
    import torch
    from paper_2206_02607_amd import crom
    D = crom.Decoder.from_layers(dec, m, precision=prec, device=cuda)
    T = crom.Trainer(D, _flat(enc), hidden, torch.from_numpy(x).to(cuda), u.shape[0])
    return D, T


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("shape", ["1d", "2d", "3d"])
def test_train_grads(cuda, shape, prec):
    import torch
    B, P = 3, (300 if shape != "3d" else 200)
    dec, enc, x, u, m = _problem(shape, 11, B, P)
    D, T = _trainer(dec, enc, x, u, m, prec, cuda)
    loss, gd, ge, q = T.grads(torch.from_numpy(u).to(cuda))
    torch.cuda.synchronize()
    rl, rgd, rge, rq = train.loss_and_grads(*_as_held(dec, enc, prec), x, u)
    if prec != "fp32":
        _, raw, _, _ = train.loss_and_grads(*_as_held(dec, enc, "fp32"), x, u)
        print("vs_fp32_weights", max(normwise_rel(g, r) for (g, _), (r, _) in zip(_split(gd.cpu().numpy(), dec), raw)),
              max(normwise_rel(g, r) for (_, g), (_, r) in zip(_split(gd.cpu().numpy(), dec), raw)))
    tol = TOL[prec]
    errs = {"loss": abs(loss.item() - rl) / rl, "q": normwise_rel(q.cpu().numpy(), rq)}
    for name, got, ref, layers in (("dec", gd, rgd, dec), ("enc", ge, rge, enc)):
        for li, ((gW, gb), (rW, rb)) in enumerate(zip(_split(got.cpu().numpy(), layers), ref)):
            errs[f"{name}W{li}"] = normwise_rel(gW, rW)
            errs[f"{name}b{li}"] = normwise_rel(gb, rb)
    print(shape, prec, {k: f"{v:.1e}" for k, v in errs.items()})
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, bad


def test_train_grads_deterministic(cuda):
    import torch
    dec, enc, x, u, m = _problem("2d", 12, 4, 257)
    D, T = _trainer(dec, enc, x, u, m, "bf16", cuda)
    ut = torch.from_numpy(u).to(cuda)
    a = [t.clone() for t in T.grads(ut)]
    b = [t.clone() for t in T.grads(ut)]
    for s, t in zip(a, b):
        assert torch.equal(s, t)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("shape", ["1d", "2d", "3d"])
def test_decode_vjp(cuda, shape, prec):
    import torch
    from paper_2206_02607_amd import crom
    m, r, d, w, depth = SHAPES[shape]
    g = rng(21)
    dec = xavier_mlp(g, m, r, d, w, depth, bias_scale=0.2)
    B, P = 2, 77
    x = uniform_points(g, P, m)
    q = g.uniform(-1, 1, size=(B, r)).astype(np.float32)
    dg = g.normal(size=(B, P, d)).astype(np.float32)
    D = crom.Decoder.from_layers(dec, m, precision=prec, device=cuda)
    gp, gq = crom.decode_vjp(D, torch.from_numpy(x).to(cuda), torch.from_numpy(q).to(cuda),
                             torch.from_numpy(dg).to(cuda))
    layers, _ = _as_held(dec, None, prec)
    a0 = np.concatenate([np.tile(x, (B, 1)), np.repeat(q, P, axis=0)], axis=1).astype(np.float64)
    _, acts = train.mlp_forward([(W.astype(np.float64), b.astype(np.float64)) for W, b in layers], a0)
    grads, d_a0 = train.mlp_backward([(W.astype(np.float64), b.astype(np.float64)) for W, b in layers], acts,
                                     dg.reshape(B * P, d).astype(np.float64))
    ref_q = d_a0[:, m:].reshape(B, P, r).sum(axis=1)
    tol = TOL[prec]
    errs = {"q": normwise_rel(gq.cpu().numpy(), ref_q)}
    for li, ((gW, gb), (rW, rb)) in enumerate(zip(_split(gp.cpu().numpy(), dec), grads)):
        errs[f"W{li}"] = normwise_rel(gW, rW)
        errs[f"b{li}"] = normwise_rel(gb, rb)
    print(shape, prec, {k: f"{v:.1e}" for k, v in errs.items()})
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, bad


def test_autograd_function_vs_oracle_and_fd(cuda):
    """The autograd wrapper's gradients equal the oracle's, and agree with a
    central difference of the fused forward kernel along a random direction."""
    import torch
    from paper_2206_02607_amd import autograd, crom
    m, r, d, w, depth = SHAPES["2d"]
    g = rng(31)
    dec = xavier_mlp(g, m, r, d, w, depth, bias_scale=0.2)
    B, P = 3, 50
    x = torch.from_numpy(uniform_points(g, P, m)).to(cuda)
    q0 = g.uniform(-1, 1, size=(B, r)).astype(np.float32)
    wts = torch.from_numpy(g.normal(size=(B, P, d)).astype(np.float32)).to(cuda)
    D = crom.Decoder.from_layers(dec, m, precision="fp32", device=cuda)
    D.params.requires_grad_(True)
    q = torch.from_numpy(q0).to(cuda).requires_grad_(True)
    G = autograd.decode(D, q, x)
    (G * wts).sum().backward()
    gp, gq = D.params.grad.detach().clone(), q.grad.detach().clone()
    # oracle
    layers = [(np.asarray(W, np.float64), np.asarray(b, np.float64))
              for W, b in _split(_flat(dec), dec)]
    xn = x.cpu().numpy().astype(np.float64)
    a0 = np.concatenate([np.tile(xn, (B, 1)), np.repeat(q0.astype(np.float64), P, axis=0)], axis=1)
    _, acts = train.mlp_forward(layers, a0)
    grads, d_a0 = train.mlp_backward(layers, acts, wts.cpu().numpy().reshape(B * P, d).astype(np.float64))
    assert normwise_rel(gq.cpu().numpy(), d_a0[:, m:].reshape(B, P, r).sum(axis=1)) <= 1e-5
    assert normwise_rel(gp.cpu().numpy(), np.concatenate([np.concatenate([a.ravel(), b.ravel()])
                                                          for a, b in grads])) <= 1e-5
    # directional central difference of the forward kernel
    v = torch.from_numpy(g.normal(size=D.params.numel()).astype(np.float32)).to(cuda)
    v /= v.norm()
    h = 1e-2
    p0 = D.params.detach().clone()
    vals = []
    for s in (h, -h):
        with torch.no_grad():
            D.params.copy_(p0 + s * v)
        D.pack()
        with torch.no_grad():
            vals.append((autograd.decode(D, q.detach(), x) * wts).sum().item())
    with torch.no_grad():
        D.params.copy_(p0)
    D.pack()
    fd = (vals[0] - vals[1]) / (2 * h)
    an = float((gp * v).sum())
    assert abs(fd - an) <= 1e-2 * max(1.0, abs(an)), (fd, an)


def test_adam_step(cuda):
    import torch
    from paper_2206_02607_amd import crom
    g = rng(41)
    n = 1000
    p = g.normal(size=n)
    ref = [p.copy()]
    opt = train.Adam(ref, lr=3e-3)
    pt = torch.from_numpy(p.astype(np.float32)).to(cuda)
    mt, vt = torch.zeros_like(pt), torch.zeros_like(pt)
    for t in range(1, 4):
        grad = g.normal(size=n) * 10.0 ** g.uniform(-4, 0, size=n)
        opt.step([grad])
        crom.adam_step(pt, torch.from_numpy(grad.astype(np.float32)).to(cuda), mt, vt, t, 3e-3)
        d_gpu = pt.cpu().numpy().astype(np.float64) - p.astype(np.float32).astype(np.float64)
        d_ref = ref[0] - p
        assert normwise_rel(d_gpu, d_ref) <= 1e-4, t


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_train_step_composes_grads_adam_pack(cuda, prec):
    """crom_train_step = crom_train_grads, then Adam on both parameter sets
    (checked against the oracle's Adam applied to the same gradients), then a
    refreshed packed copy (decoding equals a decoder built from scratch)."""
    import torch
    from paper_2206_02607_amd import crom
    dec, enc, x, u, m = _problem("2d", 51, 2, 150)
    D, T = _trainer(dec, enc, x, u, m, prec, cuda)
    ut = torch.from_numpy(u).to(cuda)
    pd0, pe0 = D.params.cpu().numpy().astype(np.float64), T.enc_params.cpu().numpy().astype(np.float64)
    _, gd, ge, _ = T.grads(ut)
    gd, ge = gd.cpu().numpy().astype(np.float64), ge.cpu().numpy().astype(np.float64)
    rd, re = [pd0.copy()], [pe0.copy()]
    train.Adam(rd, lr=1e-3).step([gd])
    train.Adam(re, lr=1e-3).step([ge])
    T.step(ut, lr=1e-3)
    torch.cuda.synchronize()
    assert normwise_rel(D.params.cpu().numpy() - pd0, rd[0] - pd0) <= 1e-4
    assert normwise_rel(T.enc_params.cpu().numpy() - pe0, re[0] - pe0) <= 1e-4
    fresh = crom.Decoder(D.params.detach().clone(), D.m, D.r, D.d, D.width, D.depth, prec, cuda)
    xs = torch.from_numpy(x).to(cuda)
    qv = torch.from_numpy(np.linspace(-1, 1, D.r)).to(cuda)
    assert torch.equal(D.decode(xs, qv), fresh.decode(xs, qv))


def test_training_trajectory_fp32(cuda):
    """Five FP32 Adam steps on the GPU follow the oracle's training loop: the
    batch loss before each step agrees to 1e-4 relative."""
    import torch
    dec, enc, x, u, m = _problem("2d", 71, 2, 150)
    D, T = _trainer(dec, enc, x, u, m, "fp32", cuda)
    ut = torch.from_numpy(u).to(cuda)
    got = [T.step(ut, lr=1e-3).item() for _ in range(5)]
    d64, e64 = [[(np.asarray(W, np.float32).astype(np.float64), np.asarray(b, np.float32).astype(np.float64))
                 for W, b in L] for L in (dec, enc)]
    opt = train.Adam(train.flatten(d64) + train.flatten(e64), lr=1e-3)
    ref = []
    for _ in range(5):
        loss, gd, ge, _ = train.loss_and_grads(d64, e64, x, u)
        ref.append(loss)
        opt.step(train.flatten(gd) + train.flatten(ge))
    print("trajectory", got, ref)
    assert np.allclose(got, ref, rtol=1e-4, atol=0)


def test_training_reduces_loss(cuda):
    """BF16 training on a smooth learnable family lowers the loss steadily."""
    import torch
    dec, enc, x, u, m = _problem("2d", 61, 4, 256)
    # u_b(x) = a_b sin(pi x0) sin(pi x1)
    amp = np.array([-0.8, -0.2, 0.4, 0.9], np.float32)
    u = (amp[:, None] * (np.sin(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1]))[None, :]).astype(np.float32)
    D, T = _trainer(dec, enc, x, u, m, "bf16", cuda)
    ut = torch.from_numpy(u).to(cuda)
    losses = [T.step(ut, lr=1e-3).item() for _ in range(300)]
    print("loss", losses[0], losses[-1])
    assert np.mean(losses[-20:]) < 0.2 * np.mean(losses[:20])


@pytest.mark.parametrize("shape", ["1d", "2d"])
def test_train_grads_siren(cuda, shape):
    """SIREN decoder (sine hidden layers; the bfloat16 row kernels store cos z
    beside sin z for the backward) with an ELU encoder, at the bfloat16-held
    weights.

    Two checks.  (1) The decoder's gradients against the oracle's reverse
    mode taken at the GPU's own latents q, to the bfloat16 tolerance 2e-2.
    (2) Loss, latents and every gradient against the oracle end to end, to
    5e-2: the latents carry the encoder's bfloat16 error (about 1.5e-3
    normwise), and the first sine layer multiplies it by weights of size up
    to omega_0 / (m + r), shifting its pre-activations by about 1e-2 rad; the
    sums over rows that form the first-layer gradients cancel by a factor of
    about 14 (sum of magnitudes over magnitude of the sum, measured on these
    inputs).  A model of the kernels' bfloat16 roundings in float64 gives
    3.6e-2 on the first bias gradient of the 1D decoder and 1.6e-2 in 2D."""
    import torch
    from paper_2206_02607_amd import crom
    from workloads import siren_mlp
    B, P = 3, 300
    m, r, d, w, depth = SHAPES[shape]
    g = rng(13)
    dec = siren_mlp(g, m, r, d, w, depth)
    enc = xavier_mlp(g, P * d, 0, r, 40, 1, bias_scale=0.2)
    x = g.uniform(-1, 1, size=(P, m))
    u = g.uniform(-1, 1, size=(B, P * d)).astype(np.float32)
    D = crom.Decoder.from_layers(dec, m, precision="bf16", device=cuda, act="sine")
    T = crom.Trainer(D, _flat(enc), 40, torch.from_numpy(x).to(cuda), B)
    loss, gd, ge, q = T.grads(torch.from_numpy(u).to(cuda))
    torch.cuda.synchronize()
    rl, rgd, rge, rq = train.loss_and_grads(*_as_held(dec, enc, "bf16"), x, u, dec_act="sine")
    errs = {"loss": abs(loss.item() - rl) / rl, "q": normwise_rel(q.cpu().numpy(), rq)}
    for name, got, ref, layers in (("dec", gd, rgd, dec), ("enc", ge, rge, enc)):
        for li, ((gW, gb), (rW, rb)) in enumerate(zip(_split(got.cpu().numpy(), layers), ref)):
            errs[f"{name}W{li}"] = normwise_rel(gW, rW)
            errs[f"{name}b{li}"] = normwise_rel(gb, rb)
    print("siren", shape, {k: f"{v:.1e}" for k, v in errs.items()})
    bad = {k: v for k, v in errs.items() if not v <= 5e-2}
    assert not bad, bad
    # (1) the decoder alone, at the latents the GPU formed
    held_dec = _as_held(dec, enc, "bf16")[0]
    qg = q.cpu().numpy().astype(np.float64)
    a0 = np.concatenate([np.tile(x, (B, 1)), np.repeat(qg, P, axis=0)], axis=1)
    out, acts = train.mlp_forward(held_dec, a0, "sine")
    resid = out - u.reshape(B * P, d).astype(np.float64)
    qgrads, _ = train.mlp_backward(held_dec, acts, (2.0 / resid.size) * resid, "sine")
    derr = {}
    for li, ((gW, gb), (rW, rb)) in enumerate(zip(_split(gd.cpu().numpy(), dec), qgrads)):
        derr[f"W{li}"] = normwise_rel(gW, rW)
        derr[f"b{li}"] = normwise_rel(gb, rb)
    print("siren decoder at the GPU latents", {k: f"{v:.1e}" for k, v in derr.items()})
    bad = {k: v for k, v in derr.items() if not v <= TOL["bf16"]}
    assert not bad, bad


def test_siren_training_reduces_loss(cuda):
    import torch
    from paper_2206_02607_amd import crom
    from workloads import siren_mlp
    B, P = 4, 256
    m, r, d, w, depth = SHAPES["2d"]
    g = rng(14)
    dec = siren_mlp(g, m, r, d, w, depth)
    enc = xavier_mlp(g, P, 0, r, 40, 1, bias_scale=0.2)
    x = g.uniform(-1, 1, size=(P, m))
    u = (np.sin(3 * x[:, 0])[None] * g.uniform(0.5, 1, size=(B, 1))).astype(np.float32)
    D = crom.Decoder.from_layers(dec, m, precision="bf16", device=cuda, act="sine")
    T = crom.Trainer(D, _flat(enc), 40, torch.from_numpy(x).to(cuda), B)
    ut = torch.from_numpy(u).to(cuda)
    losses = [T.step(ut, 1e-4)[0].item() for _ in range(200)]
    print("siren loss", losses[0], losses[-1])
    assert losses[-1] < 0.1 * losses[0]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("shape", ["2d", "3d"])
def test_train_grads_conv_encoder(cuda, shape, prec):
    """The paper's convolutional encoder (kernel 6, stride 4; 300 points:
    one convolution to 74 for d = 1, two to 18 for d = 3; dense 32): loss,
    latents and every gradient against the oracle.  The encoder's
    arithmetic is FP32 in every mode; in the bfloat16 mode its gradients
    inherit the decoder's bfloat16 latent cotangent (tolerance 2e-2)."""
    import torch
    from paper_2206_02607_amd import crom
    m, r, d, w, depth = SHAPES[shape]
    B, P = 3, 300
    g = rng(15)
    dec = xavier_mlp(g, m, r, d, w, depth, bias_scale=0.2)
    enc = train.conv_encoder_init(g, P, d, r, 32)
    x = uniform_points(g, P, m)
    u = g.uniform(-1, 1, size=(B, P * d)).astype(np.float32)
    D = crom.Decoder.from_layers(dec, m, precision=prec, device=cuda)
    assert crom.encoder_param_count(P * d, 32, r, "conv", d) == _flat(enc).size
    T = crom.Trainer(D, _flat(enc), 32, torch.from_numpy(x).to(cuda), B, enc_kind="conv")
    loss, gd, ge, q = T.grads(torch.from_numpy(u).to(cuda))
    q_only = T.encode(torch.from_numpy(u).to(cuda))
    torch.cuda.synchronize()
    held_dec, _ = _as_held(dec, None, prec)
    enc64 = [(np.asarray(W, np.float32).astype(np.float64), np.asarray(b, np.float32).astype(np.float64))
             for W, b in enc]
    rl, rgd, rge, rq = train.loss_and_grads(held_dec, enc64, x, u, enc_kind="conv")
    errs = {"loss": abs(loss.item() - rl) / rl, "q": normwise_rel(q.cpu().numpy(), rq),
            "q_encode": normwise_rel(q_only.cpu().numpy(), rq)}
    for name, got, ref, layers in (("dec", gd, rgd, dec), ("enc", ge, rge, enc)):
        for li, ((gW, gb), (rW, rb)) in enumerate(zip(_split(got.cpu().numpy(), layers), ref)):
            errs[f"{name}W{li}"] = normwise_rel(gW, rW)
            errs[f"{name}b{li}"] = normwise_rel(gb, rb)
    print(shape, prec, "conv encoder", {k: f"{v:.1e}" for k, v in errs.items()})
    assert errs["q"] <= 1e-5 and errs["q_encode"] <= 1e-5  # FP32 encoder in every mode
    bad = {k: v for k, v in errs.items() if not v <= TOL[prec]}
    assert not bad, bad


def test_conv_encoder_training_reduces_loss(cuda):
    import torch
    from paper_2206_02607_amd import crom
    m, r, d, w, depth = SHAPES["2d"]
    B, P = 4, 256
    g = rng(16)
    dec = xavier_mlp(g, m, r, d, w, depth)
    enc = train.conv_encoder_init(g, P, d, r, 32)
    x = uniform_points(g, P, m)
    amp = np.array([-0.8, -0.2, 0.4, 0.9], np.float32)
    u = (amp[:, None] * (np.sin(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1]))[None, :]).astype(np.float32)
    D = crom.Decoder.from_layers(dec, m, precision="bf16", device=cuda)
    T = crom.Trainer(D, _flat(enc), 32, torch.from_numpy(x).to(cuda), B, enc_kind="conv")
    ut = torch.from_numpy(u).to(cuda)
    losses = [T.step(ut, lr=1e-3).item() for _ in range(300)]
    print("conv encoder loss", losses[0], losses[-1])
    assert np.mean(losses[-20:]) < 0.2 * np.mean(losses[:20])


def test_conv_encoder_full_size(cuda):
    """The training workload's size: 128 x 128 = 16,384 points per snapshot
    (convolutions 16384 -> 4095 -> 1023 -> 255 -> 63, dense 32, r = 8), the
    2D decoder, FP32, two snapshots: loss, latents and every gradient
    against the oracle (1e-5)."""
    import torch
    from paper_2206_02607_amd import crom
    from workloads import grid_points_2d
    m, r, d, w, depth = SHAPES["2d"]
    B = 2
    x = grid_points_2d(128, 128)
    P = x.shape[0]
    g = rng(17)
    dec = xavier_mlp(g, m, r, d, w, depth, bias_scale=0.2)
    enc = train.conv_encoder_init(g, P, d, r, 32)
    u = (np.sin(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1]))[None, :] * g.uniform(-1, 1, size=(B, 1))
    u = (u + 0.1 * g.uniform(-1, 1, size=(B, P))).astype(np.float32)
    D = crom.Decoder.from_layers(dec, m, precision="fp32", device=cuda)
    T = crom.Trainer(D, _flat(enc), 32, torch.from_numpy(x).to(cuda), B, enc_kind="conv")
    loss, gd, ge, q = T.grads(torch.from_numpy(u).to(cuda))
    torch.cuda.synchronize()
    rl, rgd, rge, rq = train.loss_and_grads(dec, enc, x, u, enc_kind="conv")
    errs = {"loss": abs(loss.item() - rl) / rl, "q": normwise_rel(q.cpu().numpy(), rq)}
    for name, got, ref, layers in (("dec", gd, rgd, dec), ("enc", ge, rge, enc)):
        for li, ((gW, gb), (rW, rb)) in enumerate(zip(_split(got.cpu().numpy(), layers), ref)):
            errs[f"{name}W{li}"] = normwise_rel(gW, rW)
            errs[f"{name}b{li}"] = normwise_rel(gb, rb)
    print("full size conv encoder", {k: f"{v:.1e}" for k, v in errs.items()})
    bad = {k: v for k, v in errs.items() if not v <= TOL["fp32"]}
    assert not bad, bad


def test_train_grads_bf16_full_size(cuda):
    """The bfloat16 gradient step at the size the benchmark times: 16
    snapshots of the 128 x 128 nodes (262,144 decoder rows), dense encoder
    16,384 -> 256 -> 8, against the oracle at the bfloat16-held weights, 2e-2
    per tensor.  The snapshots are standardized smooth fields (products of
    sine modes with seeded amplitudes and decay factors), the shape of the
    training data."""
    import torch
    from workloads import Train2D
    w = Train2D(seed=3)
    x = w.nodes
    P = x.shape[0]
    g = rng(31)
    k = np.arange(1, 5)
    fields = []
    for _ in range(w.batch):
        a = g.uniform(-1, 1, size=(4, 4)) * np.exp(-g.uniform(0, 0.3) * (k[:, None] ** 2 + k[None, :] ** 2))
        sx = np.sin(np.pi * np.outer(x[:, 0], k))
        sy = np.sin(np.pi * np.outer(x[:, 1], k))
        fields.append(np.einsum("pk,kl,pl->p", sx, a, sy))
    u = np.stack(fields)
    u = ((u - u.mean()) / u.std()).astype(np.float32)
    xs = ((x - x.mean(axis=0)) / x.std(axis=0)).astype(np.float32)
    dec, enc = w.layers, w.enc_layers
    D, T = _trainer(dec, enc, xs, u, w.m, "bf16", cuda, hidden=w.enc_hidden)
    loss, gd, ge, q = T.grads(torch.from_numpy(u).to(cuda))
    torch.cuda.synchronize()
    rl, rgd, rge, rq = train.loss_and_grads(*_as_held(dec, enc, "bf16"), xs, u)
    errs = {"loss": abs(loss.item() - rl) / rl, "q": normwise_rel(q.cpu().numpy(), rq)}
    for name, got, ref, layers in (("dec", gd, rgd, dec), ("enc", ge, rge, enc)):
        for li, ((gW, gb), (rW, rb)) in enumerate(zip(_split(got.cpu().numpy(), layers), ref)):
            errs[f"{name}W{li}"] = normwise_rel(gW, rW)
            errs[f"{name}b{li}"] = normwise_rel(gb, rb)
    print("bf16 full size", {k: f"{v:.1e}" for k, v in errs.items()})
    bad = {k: v for k, v in errs.items() if not v <= TOL["bf16"]}
    assert not bad, bad


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_train_state_checkpoint_resume(cuda, prec):
    """The training state is one blob (crom_train_state_offsets): a run
    resumed from a copy of it and its Adam step reproduces the uninterrupted
    run bit for bit (losses, parameters, moments)."""
    import torch
    dec, enc, x, u, m = _problem("2d", 13, 4, 257)
    D, T = _trainer(dec, enc, x, u, m, prec, cuda)
    batches = [torch.from_numpy(np.roll(u, k, axis=0).copy()).to(cuda) for k in range(7)]
    for k in range(3):
        T.step(batches[k], 1e-3)
    ck = T.checkpoint()
    run_a = [T.step(batches[k], 1e-3).clone() for k in range(3, 7)]
    end_a = T.state.clone()
    packed_a = D.packed.clone()
    T.restore(ck)
    run_b = [T.step(batches[k], 1e-3).clone() for k in range(3, 7)]
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(run_a, run_b))
    assert torch.equal(end_a, T.state)
    assert torch.equal(packed_a, D.packed)
    # the blob's sections are the views the trainer and decoder use
    lay = T.layout
    nd = D.params.numel()
    assert torch.equal(T.state[lay.dec_params:lay.dec_params + 4 * nd].view(torch.float32), D.params)
    assert lay.total == len(T.state) and lay.dec_params == 0
