"""Decoder g_theta(x, q) and its derivatives in FP64 (test infrastructure only).

The decoder is the paper's manifold-parameterisation network (Sec. "Method:
Overview and Manifold Construction", Sec. "Network Details"): an MLP whose
input is the spatial coordinate x (m values) concatenated with the latent
vector q (r values), ``depth`` hidden ELU layers of equal width and a linear
output layer with d outputs.

Readings taken where the paper is silent:
* input order a_0 = [x; q] (x first); no output activation;
* ELU with alpha = 1; at z = 0 the exponential branch is taken, so
  ELU(0) = 0, ELU'(0) = 1 and ELU''(0) = 1.
* The sine activation (Sec. "Network Details" names SIREN as the
  alternative): a_l = sin(z_l), with the SIREN frequency omega_0 folded
  into the weights and biases (a layer sin(omega_0 (W a + b)) is
  sin(W' a + b') with W' = omega_0 W, b' = omega_0 b), so s' = cos and
  s'' = -sin.

Derivatives follow the forward chain rule of Alg. "Network gradient"
(Sec. "Network Gradients via Direct Differentiation"): each layer maps the
value together with its tangents, so one pass yields g, dg/dx and dg/dq.  The
pass is extended to second order in x (the heat update needs the Laplacian):
for a_l = s(z_l),
    d a_l / d u        = s'(z_l) * d z_l / d u
    d2 a_l / d u d v   = s''(z_l) * (d z_l/d u)(d z_l/d v) + s'(z_l) * d2 z_l / d u d v
and the linear maps z_l = W_l a_{l-1} + b_l carry tangents through W_l.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

Layer = Tuple[np.ndarray, np.ndarray]


def as_f64(layers: Sequence[Layer]) -> List[Layer]:
    return [(np.asarray(W, dtype=np.float64), np.asarray(b, dtype=np.float64))
            for W, b in layers]


def elu(z):
    return np.where(z > 0, z, np.expm1(np.minimum(z, 0.0)))


def elu_d1(z):
    return np.where(z > 0, 1.0, np.exp(np.minimum(z, 0.0)))


def elu_d2(z):
    return np.where(z > 0, 0.0, np.exp(np.minimum(z, 0.0)))


def sine(z):
    return np.sin(z)


def sine_d1(z):
    return np.cos(z)


def sine_d2(z):
    return -np.sin(z)


ACTIVATIONS = {"elu": (elu, elu_d1, elu_d2), "sine": (sine, sine_d1, sine_d2)}


def _inputs(x, q):
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    q = np.asarray(q, dtype=np.float64).ravel()
    return np.concatenate([x, np.broadcast_to(q, (x.shape[0], q.size))], axis=1)


def preactivations(layers: Sequence[Layer], x, q, act: str = "elu") -> List[np.ndarray]:
    """Hidden pre-activations z_1..z_H at every point (used by tests to keep
    finite-difference probes away from the ELU kink)."""
    s0 = ACTIVATIONS[act][0]
    layers = as_f64(layers)
    a = _inputs(x, q)
    zs = []
    for W, b in layers[:-1]:
        z = a @ W.T + b
        zs.append(z)
        a = s0(z)
    return zs


def decode(layers: Sequence[Layer], x, q, act: str = "elu") -> np.ndarray:
    """g(x_p, q) at every point: x [P, m], q [r] -> g [P, d]."""
    s0 = ACTIVATIONS[act][0]
    layers = as_f64(layers)
    a = _inputs(x, q)
    for W, b in layers[:-1]:
        a = s0(a @ W.T + b)
    W, b = layers[-1]
    return a @ W.T + b


def decode_jets(layers: Sequence[Layer], x, q, m: int, act: str = "elu"):
    """Value and exact derivatives by forward-mode propagation.

    Returns (g [P,d], dg/dx [P,d,m], d2g/dx2 [P,d,m,m], dg/dq [P,d,r]).
    Tangents are carried for every network input (the m coordinates and the
    r latent entries); second-order tangents for the m coordinates only.
    """
    s0, d1, d2 = ACTIVATIONS[act]
    layers = as_f64(layers)
    a = _inputs(x, q)
    P, n0 = a.shape
    # da[p, unit, input]: derivative of each unit with respect to each input.
    da = np.zeros((P, n0, n0))
    da[:, np.arange(n0), np.arange(n0)] = 1.0
    # dda[p, unit, i, j]: second derivative with respect to x_i, x_j.
    dda = np.zeros((P, n0, m, m))
    for W, b in layers[:-1]:
        z = a @ W.T + b
        dz = np.einsum("uk,pki->pui", W, da)
        ddz = np.einsum("uk,pkij->puij", W, dda)
        s1 = d1(z)
        s2 = d2(z)
        a = s0(z)
        dzx = dz[:, :, :m]
        dda = (s2[:, :, None, None] * dzx[:, :, :, None] * dzx[:, :, None, :]
               + s1[:, :, None, None] * ddz)
        da = s1[:, :, None] * dz
    W, b = layers[-1]
    g = a @ W.T + b
    dg = np.einsum("ok,pki->poi", W, da)
    ddg = np.einsum("ok,pkij->poij", W, dda)
    return g, dg[:, :, :m], ddg, dg[:, :, m:]


def laplacian(hess: np.ndarray) -> np.ndarray:
    """Sum of the diagonal second derivatives: [P,d,m,m] -> [P,d]."""
    return np.einsum("pdii->pd", hess)


def hessian_packed(hess: np.ndarray) -> np.ndarray:
    """Upper triangle of the symmetric x-Hessian, row-major over (i <= j):
    [P,d,m,m] -> [P,d,m(m+1)/2]."""
    m = hess.shape[-1]
    iu = np.triu_indices(m)
    return hess[:, :, iu[0], iu[1]]


class MLPDecoder:
    """Adapter giving the latent step the decoder quantities it needs."""

    def __init__(self, layers: Sequence[Layer], m: int, act: str = "elu"):
        self.layers = as_f64(layers)
        self.m = m
        self.act = act
        self.r = self.layers[0][0].shape[1] - m
        self.d = self.layers[-1][0].shape[0]

    def value(self, y, q):
        return decode(self.layers, y, q, self.act)

    def jac_q(self, y, q):
        return decode_jets(self.layers, y, q, self.m, self.act)[3]

    def value_jac_q(self, y, q):
        g, _, _, J = decode_jets(self.layers, y, q, self.m, self.act)
        return g, J

    def jets(self, y, q):
        return decode_jets(self.layers, y, q, self.m, self.act)

    def laplacian(self, y, q):
        return laplacian(decode_jets(self.layers, y, q, self.m, self.act)[2])
