"""The three-stage latent step in FP64 (test infrastructure only).

Alg. "Latent-space Dynamics" with Alg. "Network inference" and Alg. "Network
inversion": (1) evaluate the decoder and its derivatives at the integration
samples for q_n; (2) advance the field at the samples with the exact PDE and
an explicit integrator; (3) find q_{n+1} whose decoded field best matches the
advanced samples in least squares, starting from q_n.

``decoder`` is any object with ``value(y, q) -> [S, d]``,
``value_jac_q(y, q) -> ([S, d], [S, d, r])`` and, for the heat equation,
``laplacian(y, q) -> [S, d]`` (``oracle.mlp.MLPDecoder`` or an analytic
stand-in from ``oracle.heat``).
"""
from __future__ import annotations

import numpy as np

from .heat import rom_heat_targets
from .inversion import GNOptions, gauss_newton, gauss_newton_from_guess


def invert(decoder, y, target: np.ndarray, q0: np.ndarray, opts: GNOptions):
    """Least-squares projection of ``target`` [S, d] onto the decoder from q0."""
    def value_fn(q):
        return decoder.value(y, q).ravel()

    def value_jac_fn(q):
        g, J = decoder.value_jac_q(y, q)
        return g.ravel(), J.reshape(-1, J.shape[-1])

    return gauss_newton(value_fn, value_jac_fn, target, q0, opts)


def heat_step(decoder, y, q_n: np.ndarray, nu: float, dt: float,
              opts: GNOptions, clamp=None):
    """q_n -> q_{n+1} for u_t = nu * Laplacian(u).  Returns (q_next, info, f_next)."""
    g = decoder.value(y, q_n)
    lap = decoder.laplacian(y, q_n)
    f_next = rom_heat_targets(g, lap, nu, dt, clamp)
    q_next, info = invert(decoder, y, f_next, q_n, opts)
    return q_next, info, f_next


def heat_rollout(decoder, y, q0: np.ndarray, nu: float, dt: float, steps: int,
                 opts: GNOptions, clamp=None):
    """Repeated heat steps; returns (trajectory [steps+1, r], list of infos)."""
    qs = [np.asarray(q0, dtype=np.float64)]
    infos = []
    for _ in range(steps):
        q, info, _ = heat_step(decoder, y, qs[-1], nu, dt, opts, clamp)
        qs.append(q)
        infos.append(info)
    return np.stack(qs), infos


def heat_step_from_guess(decoder, y, q_n: np.ndarray, q_guess, nu: float, dt: float, opts: GNOptions,
                         clamp=None):
    """heat_step with a second candidate start (``gauss_newton_from_guess``).
    Returns (q_next, info, f_next, used_guess)."""
    g = decoder.value(y, q_n)
    f_next = rom_heat_targets(g, decoder.laplacian(y, q_n), nu, dt, clamp)

    def value_fn(q):
        return decoder.value(y, q).ravel()

    def value_jac_fn(q):
        gg, J = decoder.value_jac_q(y, q)
        return gg.ravel(), J.reshape(-1, J.shape[-1])

    q, info, used = gauss_newton_from_guess(value_fn, value_jac_fn, f_next, q_n, q_guess, opts)
    return q, info, f_next, used


def encoder_guess(decoder, encode_fn, nodes, q_n: np.ndarray, nu: float, dt: float) -> np.ndarray:
    """The encoder's latent for the updated field (Sec. "Initial Guess for
    the Nonlinear Solver"): the heat update g + dt nu Laplacian(g) of the
    decoded field at every node (the full-order node set, not only the
    samples), passed through the training encoder ``encode_fn`` ([B, P] ->
    [B, r])."""
    f = rom_heat_targets(decoder.value(nodes, q_n), decoder.laplacian(nodes, q_n), nu, dt)
    return np.asarray(encode_fn(f.reshape(1, -1)), dtype=np.float64)[0]
