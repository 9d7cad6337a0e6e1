"""Training of the manifold parameterisation in FP64 (test infrastructure only).

Sec. "Manifold Construction", eq. "loss": the encoder maps a snapshot
vec f(t) to a latent q = e(f); the decoder reconstructs the snapshot at every
spatial sample, and both are fitted by minimising the squared reconstruction
error.  Readings (Sec. "Training Details" leaves them open):
* loss = mean over the batch's B snapshots, P points and d output values of
  (g(x_i, q_b) - u_b(x_i))^2; a snapshot of a d-valued field is the vector
  of its P points' values, point-major ([P][d] flattened);
* encoder q = E2 ELU(E1 u + c1) + c2 (two dense layers, ELU; the training
  workload fixes a dense one), or the paper's convolutional encoder
  (``enc_kind="conv"``, readings with ``conv_lengths``);
* Adam (Kingma & Ba) with beta1 = 0.9, beta2 = 0.999, eps = 1e-8 and bias
  correction.

* a SIREN decoder (sine hidden layers, omega_0 folded into the weights)
  trains on the same loss; the encoder stays ELU.

Gradients are taken by the reverse-mode chain rule written out layer by
layer: with a_l = s(z_l), dL/dz_l = dL/da_l * s'(z_l), dL/dW_l = sum over
points of dL/dz_l a_{l-1}^T, dL/db_l = sum dL/dz_l, dL/da_{l-1} = W_l^T dL/dz_l
(s = ELU or sin, s' = ELU' or cos).
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

from .mlp import ACTIVATIONS, as_f64

Layer = Tuple[np.ndarray, np.ndarray]


def mlp_forward(layers: Sequence[Layer], a0: np.ndarray, act: str = "elu"):
    """Hidden layers (ELU or sine) and a linear output; returns (output,
    [(z_l, a_l)]) with a_0 = the input (rows are samples)."""
    s0 = ACTIVATIONS[act][0]
    acts = [(None, a0)]
    a = a0
    for W, b in layers[:-1]:
        z = a @ W.T + b
        a = s0(z)
        acts.append((z, a))
    W, b = layers[-1]
    return a @ W.T + b, acts


def mlp_backward(layers: Sequence[Layer], acts, d_out: np.ndarray, act: str = "elu"):
    """Reverse mode through mlp_forward: returns ([(dW_l, db_l)], d_input)."""
    s1 = ACTIVATIONS[act][1]
    grads: List[Layer] = [None] * len(layers)
    W, b = layers[-1]
    a_prev = acts[-1][1]
    grads[-1] = (d_out.T @ a_prev, d_out.sum(axis=0))
    d_a = d_out @ W
    for l in range(len(layers) - 2, -1, -1):
        z, _ = acts[l + 1]
        d_z = d_a * s1(z)
        a_prev = acts[l][1]
        grads[l] = (d_z.T @ a_prev, d_z.sum(axis=0))
        d_a = d_z @ layers[l][0]
    return grads, d_a


# ---------------------------------------------------------------------------
# Convolutional encoder (Sec. "Network Details"): a snapshot is a 1D vector
# of its N points with d channels; 1D convolutions of kernel 6 and stride 4
# with d output channels are applied until the length is the smallest one
# not below 32 / d; the result is flattened to one channel, a dense layer
# maps it to 32 values and a last dense layer to r.
# Readings: no padding (length L -> floor((L - 6) / 4) + 1); ELU after every
# convolution and after the 32-wide layer, the last layer linear (as the
# decoder's output); flattening is channel-major (value (c, j) at c * L + j);
# the width of the dense layer is a parameter (the paper's is 32).
# ---------------------------------------------------------------------------

CONV_K, CONV_S = 6, 4


def conv_lengths(n: int, d: int) -> List[int]:
    """Output lengths of the convolution stack for N = n points, d channels."""
    out, L = [], n
    while L >= CONV_K:
        nxt = (L - CONV_K) // CONV_S + 1
        if nxt * d < 32:
            break
        out.append(nxt)
        L = nxt
    return out


def conv1d(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[b, o, j] = b[o] + sum_{c, k} W[o, c, k] x[b, c, 4 j + k]."""
    L = x.shape[2]
    n_out = (L - CONV_K) // CONV_S + 1
    y = np.zeros((x.shape[0], W.shape[0], n_out))
    for k in range(CONV_K):
        xs = x[:, :, k:k + CONV_S * (n_out - 1) + 1:CONV_S]  # [B, C, n_out]: x[b, c, 4 j + k]
        y += np.einsum("oc,bcj->boj", W[:, :, k], xs)
    return y + b[None, :, None]


def conv1d_backward(x: np.ndarray, W: np.ndarray, dy: np.ndarray):
    """Reverse mode of conv1d: (dx, dW, db) for the output cotangent dy."""
    n_out = dy.shape[2]
    dx = np.zeros_like(x)
    dW = np.zeros_like(W)
    for k in range(CONV_K):
        sl = slice(k, k + CONV_S * (n_out - 1) + 1, CONV_S)
        dW[:, :, k] = np.einsum("boj,bcj->oc", dy, x[:, :, sl])
        dx[:, :, sl] += np.einsum("boj,oc->bcj", dy, W[:, :, k])
    return dx, dW, dy.sum(axis=(0, 2))


def conv_encoder_init(gen, n: int, d: int, r: int, hidden: int = 32) -> List[Layer]:
    """Layers [(W [d, d, 6], b [d])..., (E1 [hidden, L d], c1), (E2 [r, hidden], c2)],
    Xavier-uniform (fan_in = d * 6 for the convolutions), biases U(-0.1, 0.1)
    so that every bias path carries a value; float32."""
    layers: List[Layer] = []
    for _ in conv_lengths(n, d):
        a = np.sqrt(6.0 / (d * CONV_K + d * CONV_K))
        layers.append((gen.uniform(-a, a, size=(d, d, CONV_K)).astype(np.float32),
                       gen.uniform(-0.1, 0.1, size=d).astype(np.float32)))
    L = conv_lengths(n, d)[-1] if conv_lengths(n, d) else n
    for n_in, n_out in ((L * d, hidden), (hidden, r)):
        a = np.sqrt(6.0 / (n_in + n_out))
        layers.append((gen.uniform(-a, a, size=(n_out, n_in)).astype(np.float32),
                       gen.uniform(-0.1, 0.1, size=n_out).astype(np.float32)))
    return layers


def conv_encoder_forward(enc: Sequence[Layer], u: np.ndarray, d: int):
    """q [B, r] for snapshots u [B, N d] (point-major), and the activations."""
    enc = as_f64(enc)
    B = u.shape[0]
    x = np.asarray(u, dtype=np.float64).reshape(B, -1, d).transpose(0, 2, 1)  # [B, d, N]
    elu = ACTIVATIONS["elu"][0]
    acts = [(None, x)]
    for W, b in enc[:-2]:
        z = conv1d(x, W, b)
        x = elu(z)
        acts.append((z, x))
    flat = x.reshape(B, -1)
    q, dense_acts = mlp_forward(enc[-2:], flat)
    return q, (acts, dense_acts)


def conv_encoder_backward(enc: Sequence[Layer], state, dq: np.ndarray):
    """Gradients [(dW, db)...] of every layer for the cotangent dq [B, r]."""
    enc = as_f64(enc)
    acts, dense_acts = state
    dense_grads, d_flat = mlp_backward(enc[-2:], dense_acts, dq)
    d1 = ACTIVATIONS["elu"][1]
    x_last = acts[-1][1]
    d_a = d_flat.reshape(x_last.shape)
    grads: List[Layer] = [None] * (len(enc) - 2)
    for l in range(len(enc) - 3, -1, -1):
        z, _ = acts[l + 1]
        d_z = d_a * d1(z)
        d_a, dW, db = conv1d_backward(acts[l][1], enc[l][0], d_z)
        grads[l] = (dW, db)
    return grads + list(dense_grads)


def encode(enc: Sequence[Layer], u: np.ndarray) -> np.ndarray:
    """q [B, r] for snapshots u [B, P]."""
    q, _ = mlp_forward(as_f64(enc), np.asarray(u, dtype=np.float64))
    return q


def loss_and_grads(dec: Sequence[Layer], enc: Sequence[Layer], x: np.ndarray, u: np.ndarray,
                   dec_act: str = "elu", enc_kind: str = "dense"):
    """Reconstruction loss of eq. "loss" and its gradients.

    dec: decoder layers (input [x; q], m = x.shape[1]); enc: encoder layers
    (input the P * d snapshot values); x [P, m] points; u [B, P * d]
    snapshots, point-major.
    Returns (loss, dec_grads, enc_grads, q)."""
    dec, enc = as_f64(dec), as_f64(enc)
    x = np.asarray(x, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    B, P = u.shape[0], x.shape[0]
    d_out = dec[-1][0].shape[0]
    if enc_kind == "conv":
        q, enc_state = conv_encoder_forward(enc, u, d_out)
    else:
        q, enc_acts = mlp_forward(enc, u)
    r = q.shape[1]
    # decoder at every (snapshot, point): rows ordered snapshot-major
    a0 = np.concatenate([np.tile(x, (B, 1)), np.repeat(q, P, axis=0)], axis=1)
    g, dec_acts = mlp_forward(dec, a0, dec_act)
    resid = g - u.reshape(B * P, g.shape[1])
    loss = float(np.mean(resid ** 2))
    d_g = (2.0 / resid.size) * resid
    dec_grads, d_a0 = mlp_backward(dec, dec_acts, d_g, dec_act)
    m = x.shape[1]
    d_q = d_a0[:, m:].reshape(B, P, r).sum(axis=1)
    if enc_kind == "conv":
        enc_grads = conv_encoder_backward(enc, enc_state, d_q)
    else:
        enc_grads, _ = mlp_backward(enc, enc_acts, d_q)
    return loss, dec_grads, enc_grads, q


class Adam:
    """Adam with bias correction over a list of arrays (updated in place)."""

    def __init__(self, params: Sequence[np.ndarray], lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.params = list(params)
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [np.zeros_like(p) for p in self.params]
        self.v = [np.zeros_like(p) for p in self.params]
        self.t = 0

    def step(self, grads: Sequence[np.ndarray]):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        for p, g, m, v in zip(self.params, grads, self.m, self.v):
            m *= self.b1
            m += (1.0 - self.b1) * g
            v *= self.b2
            v += (1.0 - self.b2) * g * g
            p -= self.lr * (m / c1) / (np.sqrt(v / c2) + self.eps)


def flatten(layers: Sequence[Layer]) -> List[np.ndarray]:
    out = []
    for W, b in layers:
        out += [W, b]
    return out


# ---------------------------------------------------------------------------
# Standardization (Sec. "Training Details"): the training fields are mapped
# to zero mean and unit variance over the whole training set, and the
# spatial coordinates of the ELU networks are standardized per axis over the
# nodes.  Readings: the variance is the population variance (divide by the
# number of values, so the standardized data has variance exactly 1); one
# mean and one deviation for all field values (every output channel alike).
# After training, the two affine maps are folded into the networks so that
# the step runs in physical units:
#   g(x, q) = u_std * g_s((x - x_mean) / x_std, q) + u_mean
#   e(u)    = e_s((u - u_mean) / u_std)
# Layer 1 of the decoder absorbs the coordinate map, the output layer the
# field map, and the encoder's first layer (dense E1 or the first
# convolution) the inverse field map.
# ---------------------------------------------------------------------------

def standardization(snaps: np.ndarray, nodes: np.ndarray):
    """(u_mean, u_std, x_mean [m], x_std [m]) of the snapshot values (every
    value of every snapshot) and of the node coordinates nodes [P, m]."""
    u = np.asarray(snaps, dtype=np.float64).ravel()
    x = np.asarray(nodes, dtype=np.float64)
    u_mean = float(np.mean(u))
    u_std = float(np.sqrt(np.mean((u - u_mean) ** 2)))
    x_mean = np.mean(x, axis=0)
    x_std = np.sqrt(np.mean((x - x_mean) ** 2, axis=0))
    return u_mean, u_std, x_mean, x_std


def fold_standardization(dec: Sequence[Layer], enc: Sequence[Layer], stats, m: int,
                         enc_kind: str = "dense"):
    """Decoder and encoder layers (FP64 copies) acting on physical points and
    fields, for networks trained on standardized ones (the identities in the
    section comment above).  ``stats`` is ``standardization``'s tuple; m is
    the number of spatial inputs (the first m columns of W_1)."""
    u_mean, u_std, x_mean, x_std = stats
    x_mean = np.asarray(x_mean, dtype=np.float64)
    x_std = np.asarray(x_std, dtype=np.float64)
    dec = [(W.copy(), b.copy()) for W, b in as_f64(dec)]
    enc = [(W.copy(), b.copy()) for W, b in as_f64(enc)]
    # layer 1: W1x x_s = W1x diag(1/x_std) x - W1x (x_mean / x_std)
    W1, b1 = dec[0]
    b1 -= W1[:, :m] @ (x_mean / x_std)
    W1[:, :m] /= x_std
    # output layer: u_std (W h + b) + u_mean
    Wo, bo = dec[-1]
    dec[-1] = (Wo * u_std, bo * u_std + u_mean)
    # encoder's first layer sees (u - u_mean) / u_std: its weights divide by
    # u_std and its bias loses u_mean / u_std times the sum of each output's
    # weights (over inputs, or over input channels and taps)
    E, c = enc[0]
    if enc_kind == "conv":
        c -= (u_mean / u_std) * E.sum(axis=(1, 2))
    else:
        c -= (u_mean / u_std) * E.sum(axis=1)
    enc[0] = (E / u_std, c)
    return dec, enc
