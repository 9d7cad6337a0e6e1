"""Pins for the training oracle (no GPU): central finite differences of the
loss on sampled parameters (decoder, encoder), an independent torch.float64
autograd computation of every gradient, and Adam's first step in closed
form."""
import numpy as np
import pytest

from oracle import train
from workloads import rng, xavier_mlp


def _problem(seed=0, B=3, P=11, m=2, r=3, w=8, depth=3, enc_hidden=6, d=1):
    g = rng(seed)
    dec = [(W.astype(np.float64), b.astype(np.float64)) for W, b in xavier_mlp(g, m, r, d, w, depth, 0.3)]
    enc = [(W.astype(np.float64), b.astype(np.float64))
           for W, b in xavier_mlp(g, P * d, 0, r, enc_hidden, 1, 0.3)]
    x = g.uniform(0, 1, size=(P, m))
    u = g.uniform(-1, 1, size=(B, P * d))
    return dec, enc, x, u


@pytest.mark.parametrize("d", [1, 3])
def test_gradients_vs_central_fd(d):
    dec, enc, x, u = _problem(d=d)
    loss, dg, eg, _ = train.loss_and_grads(dec, enc, x, u)
    g = rng(5)
    h = 1e-6
    for layers, grads in ((dec, dg), (enc, eg)):
        for li in range(len(layers)):
            for which in (0, 1):
                arr = layers[li][which]
                for _ in range(3):
                    idx = tuple(g.integers(0, s) for s in arr.shape)
                    old = arr[idx]
                    arr[idx] = old + h
                    lp = train.loss_and_grads(dec, enc, x, u)[0]
                    arr[idx] = old - h
                    lm = train.loss_and_grads(dec, enc, x, u)[0]
                    arr[idx] = old
                    fd = (lp - lm) / (2 * h)
                    assert abs(grads[li][which][idx] - fd) <= 1e-6 * max(1.0, abs(fd)), (li, which, idx)


@pytest.mark.parametrize("d", [1, 3])
def test_gradients_vs_autograd_float64(d):
    torch = pytest.importorskip("torch")
    dec, enc, x, u = _problem(seed=1, B=2, P=7, d=d)
    loss, dg, eg, q = train.loss_and_grads(dec, enc, x, u)
    T = lambda a: torch.tensor(a, dtype=torch.float64, requires_grad=True)  # noqa: E731
    tdec = [(T(W), T(b)) for W, b in dec]
    tenc = [(T(W), T(b)) for W, b in enc]

    def mlp(layers, a):
        for W, b in layers[:-1]:
            a = torch.nn.functional.elu(a @ W.T + b)
        return a @ layers[-1][0].T + layers[-1][1]

    tu = torch.tensor(u)
    tq = mlp(tenc, tu)
    B, P = u.shape[0], x.shape[0]
    a0 = torch.cat([torch.tensor(x).repeat(B, 1), tq.repeat_interleave(P, dim=0)], dim=1)
    tg = mlp(tdec, a0)
    tl = ((tg - tu.reshape(B * P, -1)) ** 2).mean()
    tl.backward()
    assert abs(tl.item() - loss) <= 1e-14 * max(1.0, loss)
    np.testing.assert_allclose(tq.detach().numpy(), q, rtol=1e-13, atol=1e-15)
    for (W, b), (gW, gb) in zip(tdec + tenc, dg + eg):
        np.testing.assert_allclose(W.grad.numpy(), gW, rtol=1e-11, atol=1e-14)
        np.testing.assert_allclose(b.grad.numpy(), gb, rtol=1e-11, atol=1e-14)


def test_adam_first_step_closed_form():
    # After one step from m = v = 0: delta = -lr * g / (|g| + eps) elementwise.
    p = np.array([1.0, -2.0, 0.5, 0.0])
    g = np.array([0.3, -1e-3, 2.0, 0.0])
    opt = train.Adam([p], lr=1e-3)
    opt.step([g])
    expect = np.array([1.0, -2.0, 0.5, 0.0]) - 1e-3 * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(p, expect, rtol=1e-12, atol=1e-15)


def test_adam_second_step_by_hand():
    p = np.array([0.2])
    opt = train.Adam([p], lr=0.1)
    opt.step([np.array([1.0])])
    opt.step([np.array([-3.0])])
    m1, v1 = 0.1 * 1.0, 0.001 * 1.0
    m2, v2 = 0.9 * m1 + 0.1 * -3.0, 0.999 * v1 + 0.001 * 9.0
    p1 = 0.2 - 0.1 * (m1 / 0.1) / (np.sqrt(v1 / 0.001) + 1e-8)
    p2 = p1 - 0.1 * (m2 / (1 - 0.81)) / (np.sqrt(v2 / (1 - 0.999 ** 2)) + 1e-8)
    np.testing.assert_allclose(p, [p2], rtol=1e-13)


def test_training_reduces_loss():
    # Fitting a family of sine snapshots: a few hundred Adam steps lower the
    # reconstruction loss (the optimisation itself, not a parity claim).
    g = rng(7)
    P, m, r = 24, 1, 2
    x = np.linspace(0, 1, P)[:, None]
    amps = g.uniform(-1, 1, size=(8, 2))
    u = amps[:, :1] * np.sin(np.pi * x[:, 0]) + amps[:, 1:] * np.sin(2 * np.pi * x[:, 0])
    dec = [(W.astype(np.float64), b.astype(np.float64)) for W, b in xavier_mlp(g, m, r, 1, 16, 3)]
    enc = [(W.astype(np.float64), b.astype(np.float64)) for W, b in xavier_mlp(g, P, 0, r, 16, 1)]
    opt = train.Adam(train.flatten(dec) + train.flatten(enc), lr=3e-3)
    l0 = train.loss_and_grads(dec, enc, x, u)[0]
    for _ in range(300):
        loss, dg, eg, _ = train.loss_and_grads(dec, enc, x, u)
        opt.step(train.flatten(dg) + train.flatten(eg))
    assert loss < 0.2 * l0


def _siren_problem(seed=2, B=2, P=7, m=2, r=3, w=8, depth=3, enc_hidden=6):
    from workloads import siren_mlp
    g = rng(seed)
    dec = [(W.astype(np.float64), b.astype(np.float64)) for W, b in siren_mlp(g, m, r, 1, w, depth)]
    enc = [(W.astype(np.float64), b.astype(np.float64)) for W, b in xavier_mlp(g, P, 0, r, enc_hidden, 1, 0.3)]
    x = g.uniform(-1, 1, size=(P, m))
    u = g.uniform(-1, 1, size=(B, P))
    return dec, enc, x, u


def test_siren_gradients_vs_central_fd():
    dec, enc, x, u = _siren_problem()
    loss, dg, eg, _ = train.loss_and_grads(dec, enc, x, u, dec_act="sine")
    g = rng(6)
    h = 1e-6
    for layers, grads in ((dec, dg), (enc, eg)):
        for li in range(len(layers)):
            for which in (0, 1):
                arr = layers[li][which]
                for _ in range(3):
                    idx = tuple(g.integers(0, s) for s in arr.shape)
                    old = arr[idx]
                    arr[idx] = old + h
                    lp = train.loss_and_grads(dec, enc, x, u, dec_act="sine")[0]
                    arr[idx] = old - h
                    lm = train.loss_and_grads(dec, enc, x, u, dec_act="sine")[0]
                    arr[idx] = old
                    fd = (lp - lm) / (2 * h)
                    assert abs(grads[li][which][idx] - fd) <= 1e-6 * max(1.0, abs(fd)), (li, which, idx)


def test_siren_gradients_vs_autograd_float64():
    torch = pytest.importorskip("torch")
    dec, enc, x, u = _siren_problem(seed=3)
    loss, dg, eg, q = train.loss_and_grads(dec, enc, x, u, dec_act="sine")
    T = lambda a: torch.tensor(a, dtype=torch.float64, requires_grad=True)  # noqa: E731
    tdec = [(T(W), T(b)) for W, b in dec]
    tenc = [(T(W), T(b)) for W, b in enc]

    def mlp(layers, a, act):
        for W, b in layers[:-1]:
            a = act(a @ W.T + b)
        return a @ layers[-1][0].T + layers[-1][1]

    tu = torch.tensor(u)
    tq = mlp(tenc, tu, torch.nn.functional.elu)
    B, P = u.shape[0], x.shape[0]
    a0 = torch.cat([torch.tensor(x).repeat(B, 1), tq.repeat_interleave(P, dim=0)], dim=1)
    tl = ((mlp(tdec, a0, torch.sin) - tu.reshape(B * P, -1)) ** 2).mean()
    tl.backward()
    assert abs(tl.item() - loss) <= 1e-14 * max(1.0, loss)
    for (W, b), (gW, gb) in zip(tdec + tenc, dg + eg):
        np.testing.assert_allclose(W.grad.numpy(), gW, rtol=1e-10, atol=1e-13)
        np.testing.assert_allclose(b.grad.numpy(), gb, rtol=1e-10, atol=1e-13)


# ---------------------------------------------------------------------------
# Convolutional encoder
# ---------------------------------------------------------------------------

def test_conv_lengths_follow_the_rule():
    # 16,384 points, one channel: 16384 -> 4095 -> 1023 -> 255 -> 63 (the
    # next, 15, would fall below 32)
    assert train.conv_lengths(16384, 1) == [4095, 1023, 255, 63]
    # three channels: down to 15 (45 values), not 3 (9 values)
    assert train.conv_lengths(16384, 3) == [4095, 1023, 255, 63, 15]
    # 40 points: one convolution would already leave 9 < 32 values
    assert train.conv_lengths(40, 1) == []


def test_conv1d_against_torch():
    torch = pytest.importorskip("torch")
    g = rng(31)
    x = g.normal(size=(3, 2, 53))
    W = g.normal(size=(2, 2, 6))
    b = g.normal(size=2)
    y = train.conv1d(x, W, b)
    tx = torch.tensor(x, requires_grad=True)
    tW = torch.tensor(W, requires_grad=True)
    tb = torch.tensor(b, requires_grad=True)
    ty = torch.nn.functional.conv1d(tx, tW, tb, stride=4)
    np.testing.assert_allclose(y, ty.detach().numpy(), rtol=1e-13, atol=1e-13)
    dy = g.normal(size=y.shape)
    ty.backward(torch.tensor(dy))
    dx, dW, db = train.conv1d_backward(x, W, dy)
    np.testing.assert_allclose(dx, tx.grad.numpy(), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(dW, tW.grad.numpy(), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(db, tb.grad.numpy(), rtol=1e-12, atol=1e-13)


def _conv_problem(seed=3, B=2, P=300, m=2, r=3, w=8, depth=3, d=1):
    g = rng(seed)
    dec = [(W.astype(np.float64), b.astype(np.float64)) for W, b in xavier_mlp(g, m, r, d, w, depth, 0.3)]
    enc = [(W.astype(np.float64), b.astype(np.float64)) for W, b in train.conv_encoder_init(g, P, d, r, 7)]
    x = g.uniform(0, 1, size=(P, m))
    u = g.uniform(-1, 1, size=(B, P * d))
    return dec, enc, x, u


@pytest.mark.parametrize("d", [1, 3])
def test_conv_encoder_gradients_vs_autograd_float64(d):
    torch = pytest.importorskip("torch")
    dec, enc, x, u = _conv_problem(d=d)
    loss, dg, eg, q = train.loss_and_grads(dec, enc, x, u, enc_kind="conv")
    T = lambda a: torch.tensor(a, dtype=torch.float64, requires_grad=True)  # noqa: E731
    tdec = [(T(W), T(b)) for W, b in dec]
    tenc = [(T(W), T(b)) for W, b in enc]
    F = torch.nn.functional
    B, P = u.shape[0], x.shape[0]
    tu = torch.tensor(u)
    a = tu.reshape(B, P, d).permute(0, 2, 1)
    for W, b in tenc[:-2]:
        a = F.elu(F.conv1d(a, W, b, stride=4))
    h = F.elu(a.reshape(B, -1) @ tenc[-2][0].T + tenc[-2][1])
    tq = h @ tenc[-1][0].T + tenc[-1][1]
    a0 = torch.cat([torch.tensor(x).repeat(B, 1), tq.repeat_interleave(P, dim=0)], dim=1)
    z = a0
    for W, b in tdec[:-1]:
        z = F.elu(z @ W.T + b)
    tg = z @ tdec[-1][0].T + tdec[-1][1]
    tl = ((tg - tu.reshape(B * P, -1)) ** 2).mean()
    tl.backward()
    assert abs(tl.item() - loss) <= 1e-14 * max(1.0, loss)
    np.testing.assert_allclose(tq.detach().numpy(), q, rtol=1e-13, atol=1e-15)
    assert len(eg) == len(train.conv_lengths(P, d)) + 2
    for (W, b), (gW, gb) in zip(tdec + tenc, dg + eg):
        np.testing.assert_allclose(W.grad.numpy(), gW, rtol=1e-11, atol=1e-14)
        np.testing.assert_allclose(b.grad.numpy(), gb, rtol=1e-11, atol=1e-14)


def test_conv_encoder_gradients_vs_central_fd():
    dec, enc, x, u = _conv_problem(seed=4, d=3)
    loss, dg, eg, _ = train.loss_and_grads(dec, enc, x, u, enc_kind="conv")
    g = rng(6)
    h = 1e-6
    for li in range(len(enc)):
        for which in (0, 1):
            arr = enc[li][which]
            for _ in range(3):
                idx = tuple(g.integers(0, s) for s in arr.shape)
                old = arr[idx]
                arr[idx] = old + h
                lp = train.loss_and_grads(dec, enc, x, u, enc_kind="conv")[0]
                arr[idx] = old - h
                lm = train.loss_and_grads(dec, enc, x, u, enc_kind="conv")[0]
                arr[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(eg[li][which][idx] - fd) <= 1e-6 * max(1.0, abs(fd)), (li, which, idx)
