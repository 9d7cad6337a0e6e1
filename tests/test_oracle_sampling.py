"""Pins for the robust-sampling oracle (no GPU).

A decoder that is linear in the latent, g(x, q) = sum_k q_k phi_k(x) with
phi_k(x) = x^k (1 - x), makes the linearised heat step a fixed linear map:
q+ = q + dt nu pinv(Phi_M) Phi''_M q, so the final latent after N steps is
(I + dt nu pinv(Phi_M) Phi''_M)^N q0 and the residual vector of a sample set
follows from a pseudo-inverse and a matrix power, without the Gauss-Newton
code the oracle runs.  Brute force over every candidate then fixes each
greedy choice."""
import numpy as np
import pytest

from oracle import heat, sampling
from oracle.inversion import GNOptions
from workloads import rng


class _PolyModes:
    """g(x, q) = sum_k q_k x^k (1 - x), k = 1..r, with its exact Laplacian."""

    def __init__(self, r):
        self.r, self.m, self.d = r, 1, 1
        self.k = np.arange(1, r + 1)

    def basis(self, y):
        x = np.asarray(y, dtype=np.float64).reshape(-1, 1)
        k = self.k[None, :]
        phi = x ** k * (1.0 - x)
        d2 = k * (k - 1) * x ** np.maximum(k - 2, 0) - (k + 1) * k * x ** (k - 1)
        return phi, d2

    def value(self, y, q):
        return (self.basis(y)[0] @ np.asarray(q, dtype=np.float64))[:, None]

    def value_jac_q(self, y, q):
        B = self.basis(y)[0]
        return (B @ q)[:, None], B[:, None, :]

    def laplacian(self, y, q):
        return (self.basis(y)[1] @ np.asarray(q, dtype=np.float64))[:, None]


P, R, N_STEPS, DT = 21, 3, 20, 1e-3
NUS = (0.5, 1.0)


def _case(seed=0):
    g = rng(seed)
    nodes = (np.arange(P) / (P - 1.0))[:, None]
    dec = _PolyModes(R)
    q0 = g.uniform(-1, 1, size=(len(NUS), R))
    a = g.uniform(-1, 1, size=3)
    ref = np.stack([heat.heat1d_modes(a, nu, N_STEPS * DT, nodes) for nu in NUS])
    return dec, nodes, q0, ref


def _closed_form_residual(dec, nodes, q0, ref, samples):
    phi_all = dec.basis(nodes)[0]
    phi, d2 = dec.basis(nodes[np.asarray(samples)])
    res = np.zeros(P)
    for k, nu in enumerate(NUS):
        T = np.eye(R) + DT * nu * np.linalg.pinv(phi) @ d2
        q = np.linalg.matrix_power(T, N_STEPS) @ q0[k]
        res += np.abs(phi_all @ q - ref[k])
    return res


def _final_latent(dec, nodes, q0, linearized):
    opts = GNOptions(max_iter=1 if linearized else 5, linearized=linearized, tol_step=1e-14)
    return sampling.heat_final_latent(dec, nodes, q0, NUS, DT, N_STEPS, opts)


def test_metric_is_mean_plus_max():
    assert sampling.metric(np.array([1.0, 2.0, 6.0])) == 9.0


def test_rank_rules():
    res = np.array([1.0, 5.0, 3.0, 5.0, np.nan, 0.0])
    assert sampling.max_indices(res, [], 3) == [4, 1, 3]
    assert sampling.max_indices(res, [4, 1], 3) == [3, 2, 0]
    assert sampling.min_index([2.0, 1.0, 1.0, np.nan]) == 1
    assert sampling.min_index([np.nan, 3.0]) == 1


@pytest.mark.parametrize("linearized", [True, False])
def test_residual_matches_matrix_power(linearized):
    dec, nodes, q0, ref = _case()
    fl = _final_latent(dec, nodes, q0, linearized)
    for samples in ([2, 9, 17], [1, 5, 11, 19], [3, 4, 5, 6, 15]):
        got = sampling.residual(dec, nodes, ref, samples, fl)
        want = _closed_form_residual(dec, nodes, q0, ref, samples)
        np.testing.assert_allclose(got, want, rtol=1e-10, atol=1e-12)


def test_residual_depends_on_the_samples():
    """Phi'' is not in the span of Phi, so the projected dynamics change with
    the sample set (the greedy loop has something to choose)."""
    dec, nodes, q0, ref = _case()
    a = _closed_form_residual(dec, nodes, q0, ref, [2, 9, 17])
    b = _closed_form_residual(dec, nodes, q0, ref, [3, 4, 5])
    assert np.abs(a - b).max() > 1e-3 * np.abs(a).max()


def test_greedy_over_all_candidates_is_brute_force():
    dec, nodes, q0, ref = _case(1)
    fl = _final_latent(dec, nodes, q0, True)
    init = [1, 10, 19]
    out = sampling.robust_sampling(dec, nodes, ref, init, fl, target=0.0, n_try=P, max_samples=7)
    M = list(init)
    for rnd in range(4):
        best = min((c for c in range(P) if c not in M),
                   key=lambda c: sampling.metric(_closed_form_residual(dec, nodes, q0, ref, M + [c])))
        assert out.samples[len(M)] == best, f"round {rnd}"
        M.append(best)
    assert out.samples == M and not out.reached
    np.testing.assert_allclose(out.metric, sampling.metric(_closed_form_residual(dec, nodes, q0, ref, M)),
                               rtol=1e-10)


def test_single_candidate_takes_largest_residual():
    dec, nodes, q0, ref = _case(2)
    fl = _final_latent(dec, nodes, q0, True)
    init = [4, 12, 16]
    out = sampling.robust_sampling(dec, nodes, ref, init, fl, target=0.0, n_try=1, max_samples=6)
    M = list(init)
    for _ in range(3):
        res = _closed_form_residual(dec, nodes, q0, ref, M)
        res[M] = -np.inf
        M.append(int(np.argmax(res)))
    assert out.samples == M


def test_candidates_are_the_top_residuals_outside_the_set():
    dec, nodes, q0, ref = _case(3)
    fl = _final_latent(dec, nodes, q0, True)
    init = [0, 7, 14]
    out = sampling.robust_sampling(dec, nodes, ref, init, fl, target=0.0, n_try=4, max_samples=6)
    M = list(init)
    for cand, mets in zip(out.candidates, out.metrics):
        res = _closed_form_residual(dec, nodes, q0, ref, M)
        outside = [i for i in range(P) if i not in M]
        want = sorted(outside, key=lambda i: (-res[i], i))[:4]
        assert cand == want
        want_m = [sampling.metric(_closed_form_residual(dec, nodes, q0, ref, M + [c])) for c in cand]
        np.testing.assert_allclose(mets, want_m, rtol=1e-10)
        M.append(cand[int(np.argmin(mets))])
    assert out.samples == M


def test_stops_at_target_and_at_size_limit():
    dec, nodes, q0, ref = _case(4)
    fl = _final_latent(dec, nodes, q0, True)
    init = [2, 8, 13]
    m0 = sampling.metric(_closed_form_residual(dec, nodes, q0, ref, init))
    out = sampling.robust_sampling(dec, nodes, ref, init, fl, target=m0 * 1.0001, n_try=3)
    assert out.reached and out.samples == init and out.candidates == []
    full = sampling.robust_sampling(dec, nodes, ref, init, fl, target=0.0, n_try=3, max_samples=6)
    assert len(full.samples) == 6 and not full.reached
    # a target just above the 5-sample metric stops at the first prefix below it
    ms = [sampling.metric(_closed_form_residual(dec, nodes, q0, ref, full.samples[:n])) for n in (3, 4, 5)]
    t = ms[2] * (1 + 1e-9)
    stop = next(n for n, m in zip((3, 4, 5), ms) if m < t)
    out = sampling.robust_sampling(dec, nodes, ref, init, fl, target=t, n_try=3)
    assert out.reached and out.samples == full.samples[:stop]
    assert len(out.candidates) == stop - 3
