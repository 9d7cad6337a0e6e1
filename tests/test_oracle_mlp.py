"""Pins for the decoder oracle: closed forms, finite differences and an
independent autograd witness (no GPU)."""
import numpy as np
import pytest

from oracle import mlp
from workloads import rng, xavier_mlp


def _rand_net(seed, m, r, d, width, depth, bias=0.3):
    return mlp.as_f64(xavier_mlp(rng(seed), m, r, d, width, depth, bias_scale=bias))


def test_affine_regime_closed_form():
    # Non-negative weights and a large first bias keep every unit in the
    # linear branch, so the network is the product of its weight matrices.
    g = rng(1)
    m, r, d = 2, 3, 2
    sizes = [m + r, 7, 5, 4, d]
    layers = []
    for i, (a, b) in enumerate(zip(sizes[:-1], sizes[1:])):
        W = g.uniform(0.1, 1.0, size=(b, a))
        bias = g.uniform(0.0, 0.5, size=b) + (10.0 if i == 0 else 0.0)
        layers.append((W, bias))
    x = g.uniform(0, 1, size=(6, m))
    q = g.uniform(0, 1, size=r)
    Wp = np.eye(m + r)
    c = np.zeros(m + r)
    aff_W, aff_b = np.eye(m + r), np.zeros(m + r)
    for W, b in layers:
        aff_W, aff_b = W @ aff_W, W @ aff_b + b
    a0 = np.concatenate([x, np.broadcast_to(q, (6, r))], axis=1)
    expect = a0 @ aff_W.T + aff_b
    gv, gx, hx, gq = mlp.decode_jets(layers, x, q, m)
    np.testing.assert_allclose(mlp.decode(layers, x, q), expect, rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(gv, expect, rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(gx, np.broadcast_to(aff_W[:, :m], (6, d, m)), rtol=1e-13)
    np.testing.assert_allclose(gq, np.broadcast_to(aff_W[:, m:], (6, d, r)), rtol=1e-13)
    assert np.all(hx == 0.0)


def test_negative_regime_closed_form():
    # One hidden layer held in the exponential branch:
    # g = w . (exp(z) - 1) + b_out, z = W1 [x; q] + b1 < 0, so
    # dg/da0_i = sum_j w_j e^{z_j} W1[j, i] and
    # d2g/dx_i dx_k = sum_j w_j e^{z_j} W1[j, i] W1[j, k].
    g = rng(2)
    m, r = 3, 2
    W1 = g.uniform(-1, 1, size=(9, m + r))
    b1 = -10.0 * np.ones(9)
    w = g.uniform(-1, 1, size=(1, 9))
    bo = np.array([0.7])
    layers = [(W1, b1), (w, bo)]
    x = g.uniform(0, 1, size=(4, m))
    q = g.uniform(-1, 1, size=r)
    a0 = np.concatenate([x, np.broadcast_to(q, (4, r))], axis=1)
    z = a0 @ W1.T + b1
    assert np.all(z < 0)
    e = np.exp(z)
    val = (np.expm1(z) * w[0]).sum(1) + 0.7
    grad = (e * w[0]) @ W1
    hess = np.einsum("pj,ji,jk->pik", e * w[0], W1[:, :m], W1[:, :m])
    gv, gx, hx, gq = mlp.decode_jets(layers, x, q, m)
    np.testing.assert_allclose(gv[:, 0], val, rtol=1e-13)
    np.testing.assert_allclose(gx[:, 0], grad[:, :m], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(gq[:, 0], grad[:, m:], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(hx[:, 0], hess, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(mlp.laplacian(hx)[:, 0], np.trace(hess, axis1=1, axis2=2), rtol=1e-12)


def test_input_order_x_first():
    # Zeroing the first m input columns of W1 must make g independent of x.
    layers = _rand_net(3, 2, 4, 1, 16, 3)
    W1, b1 = layers[0]
    W1 = W1.copy()
    W1[:, :2] = 0.0
    layers[0] = (W1, b1)
    g = rng(4)
    x = g.uniform(0, 1, size=(5, 2))
    q = g.uniform(-1, 1, size=4)
    gv, gx, hx, gq = mlp.decode_jets(layers, x, q, 2)
    assert np.all(gx == 0) and np.all(hx == 0)
    np.testing.assert_allclose(gv, gv[0:1].repeat(5, 0), rtol=1e-14)
    assert np.abs(gq).max() > 1e-3


def _away_from_kinks(layers, x, q, margin=1e-3):
    zs = mlp.preactivations(layers, x, q)
    return np.all(np.concatenate([np.abs(z) for z in zs], axis=1) > margin, axis=1)


@pytest.mark.parametrize("m,r,d,width,depth", [(1, 3, 1, 32, 5), (2, 8, 1, 24, 5), (3, 4, 3, 20, 6)])
def test_first_derivatives_vs_central_fd(m, r, d, width, depth):
    layers = _rand_net(10 + m, m, r, d, width, depth)
    g = rng(20 + m)
    x = g.uniform(0, 1, size=(12, m))
    q = g.uniform(-1, 1, size=r)
    keep = _away_from_kinks(layers, x, q)
    assert keep.sum() >= 3
    x = x[keep]
    gv, gx, hx, gq = mlp.decode_jets(layers, x, q, m)
    h = 1e-6
    for i in range(m):
        e = np.zeros(m); e[i] = h
        fd = (mlp.decode(layers, x + e, q) - mlp.decode(layers, x - e, q)) / (2 * h)
        np.testing.assert_allclose(gx[:, :, i], fd, rtol=1e-7, atol=1e-8)
    for k in range(r):
        e = np.zeros(r); e[k] = h
        fd = (mlp.decode(layers, x, q + e) - mlp.decode(layers, x, q - e)) / (2 * h)
        np.testing.assert_allclose(gq[:, :, k], fd, rtol=1e-7, atol=1e-8)


@pytest.mark.parametrize("m,r,d,width,depth", [(1, 3, 1, 32, 5), (2, 8, 1, 24, 5), (3, 4, 3, 20, 6)])
def test_second_derivatives_vs_fd(m, r, d, width, depth):
    # Central differences of the (separately pinned) first derivatives, and
    # a plain second difference of values on a small net.
    layers = _rand_net(30 + m, m, r, d, width, depth)
    g = rng(40 + m)
    x = g.uniform(0, 1, size=(40, m))
    q = g.uniform(-1, 1, size=r)
    keep = _away_from_kinks(layers, x, q, margin=1e-3)
    assert keep.sum() >= 3
    x = x[keep]
    gv, gx, hx, gq = mlp.decode_jets(layers, x, q, m)
    h = 1e-6
    for k in range(m):
        ek = np.zeros(m); ek[k] = h
        fd = (mlp.decode_jets(layers, x + ek, q, m)[1] - mlp.decode_jets(layers, x - ek, q, m)[1]) / (2 * h)
        np.testing.assert_allclose(hx[:, :, :, k], fd, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(hx, np.swapaxes(hx, 2, 3), rtol=0, atol=1e-15)
    small = _rand_net(60 + m, m, r, d, 6, 2)
    xs = g.uniform(0, 1, size=(40, m))
    xs = xs[_away_from_kinks(small, xs, q, margin=1e-2)]
    assert len(xs) >= 3
    hs = mlp.decode_jets(small, xs, q, m)[2]
    h = 1e-4
    for i in range(m):
        for k in range(m):
            ei = np.zeros(m); ei[i] = h
            ek = np.zeros(m); ek[k] = h
            fd = (mlp.decode(small, xs + ei + ek, q) - mlp.decode(small, xs + ei - ek, q)
                  - mlp.decode(small, xs - ei + ek, q) + mlp.decode(small, xs - ei - ek, q)) / (4 * h * h)
            np.testing.assert_allclose(hs[:, :, i, k], fd, rtol=1e-5, atol=1e-6)


def test_autograd_witness_float64():
    torch = pytest.importorskip("torch")
    m, r, d = 2, 5, 2
    layers = _rand_net(50, m, r, d, 16, 4)
    g = rng(51)
    x = g.uniform(0, 1, size=(3, m))
    q = g.uniform(-1, 1, size=r)
    Ws = [(torch.tensor(W), torch.tensor(b)) for W, b in layers]

    def net(inp):
        a = inp
        for W, b in Ws[:-1]:
            a = torch.nn.functional.elu(a @ W.T + b)
        return a @ Ws[-1][0].T + Ws[-1][1]

    gv, gx, hx, gq = mlp.decode_jets(layers, x, q, m)
    for p in range(3):
        a0 = torch.tensor(np.concatenate([x[p], q]))
        jac = torch.autograd.functional.jacobian(net, a0).numpy()
        np.testing.assert_allclose(jac[:, :m], gx[p], rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(jac[:, m:], gq[p], rtol=1e-12, atol=1e-14)
        for o in range(d):
            H = torch.autograd.functional.hessian(lambda v: net(v)[o], a0).numpy()
            np.testing.assert_allclose(H[:m, :m], hx[p, o], rtol=1e-10, atol=1e-13)


def test_elu_tie_reading():
    z = np.array([-1.0, 0.0, 2.0])
    np.testing.assert_array_equal(mlp.elu(z), [np.expm1(-1.0), 0.0, 2.0])
    np.testing.assert_array_equal(mlp.elu_d1(z), [np.exp(-1.0), 1.0, 1.0])
    np.testing.assert_array_equal(mlp.elu_d2(z), [np.exp(-1.0), 1.0, 0.0])


# ---- sine activation (SIREN) -------------------------------------------------

def test_sine_one_layer_closed_form():
    """g = sum_u w_u sin(A_u [x; q] + c_u) + b: gradient, Hessian and latent
    Jacobian written out (cos and -sin of the pre-activations)."""
    from workloads import siren_mlp
    g = rng(21)
    m, r = 2, 3
    layers = siren_mlp(g, m, r, 1, 16, 1)
    x = g.uniform(-1, 1, size=(7, m))
    q = g.uniform(-1, 1, size=r)
    A, c = [np.asarray(t, np.float64) for t in layers[0]]
    w, b = [np.asarray(t, np.float64) for t in layers[1]]
    z = np.concatenate([x, np.tile(q, (7, 1))], axis=1) @ A.T + c
    val, gx, hx, gq = mlp.decode_jets(layers, x, q, m, act="sine")
    np.testing.assert_allclose(val[:, 0], np.sin(z) @ w[0] + b[0], rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(gx[:, 0], (np.cos(z) * w[0]) @ A[:, :m], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(gq[:, 0], (np.cos(z) * w[0]) @ A[:, m:], rtol=1e-12, atol=1e-12)
    H = -np.einsum("pu,u,ui,uj->pij", np.sin(z), w[0], A[:, :m], A[:, :m])
    np.testing.assert_allclose(hx[:, 0], H, rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(mlp.laplacian(hx)[:, 0], np.trace(H, axis1=1, axis2=2), rtol=1e-11, atol=1e-11)


def test_sine_autograd_witness_float64():
    torch = pytest.importorskip("torch")
    from workloads import siren_mlp
    g = rng(22)
    m, r, d = 2, 3, 2
    layers = siren_mlp(g, m, r, d, 12, 3)
    x = g.uniform(-1, 1, size=(4, m))
    q = g.uniform(-1, 1, size=r)
    Ws = [(torch.tensor(W, dtype=torch.float64), torch.tensor(b, dtype=torch.float64)) for W, b in layers]

    def net(a):
        for W, b in Ws[:-1]:
            a = torch.sin(a @ W.T + b)
        W, b = Ws[-1]
        return a @ W.T + b

    val, gx, hx, gq = mlp.decode_jets(layers, x, q, m, act="sine")
    for p in range(x.shape[0]):
        a0 = torch.tensor(np.concatenate([x[p], q]))
        np.testing.assert_allclose(val[p], net(a0).detach().numpy(), rtol=1e-12, atol=1e-12)
        jac = torch.autograd.functional.jacobian(net, a0).numpy()
        np.testing.assert_allclose(gx[p], jac[:, :m], rtol=1e-10, atol=1e-10)
        np.testing.assert_allclose(gq[p], jac[:, m:], rtol=1e-10, atol=1e-10)
        for o in range(d):
            Hh = torch.autograd.functional.hessian(lambda v: net(v)[o], a0).numpy()
            np.testing.assert_allclose(hx[p, o], Hh[:m, :m], rtol=1e-9, atol=1e-9)


def test_sine_derivatives_vs_central_fd():
    """Smooth everywhere: no kink to avoid."""
    from workloads import siren_mlp
    g = rng(23)
    m, r = 2, 4
    layers = siren_mlp(g, m, r, 1, 16, 3)
    x = g.uniform(-1, 1, size=(5, m))
    q = g.uniform(-1, 1, size=r)
    _, gx, hx, _ = mlp.decode_jets(layers, x, q, m, act="sine")
    h = 1e-5
    for i in range(m):
        e = np.zeros(m)
        e[i] = h
        fd = (mlp.decode(layers, x + e, q, "sine") - mlp.decode(layers, x - e, q, "sine")) / (2 * h)
        np.testing.assert_allclose(gx[:, :, i], fd, rtol=1e-6, atol=1e-6 * np.abs(fd).max())
        gp = mlp.decode_jets(layers, x + e, q, m, act="sine")[1]
        gm = mlp.decode_jets(layers, x - e, q, m, act="sine")[1]
        np.testing.assert_allclose(hx[:, :, :, i], (gp - gm) / (2 * h), rtol=1e-5,
                                   atol=1e-6 * np.abs(hx).max())
