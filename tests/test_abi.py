"""The C-ABI library loads, exports every entry point the header declares,
and rejects bad arguments on the host before touching a GPU (no GPU)."""
import ctypes

import numpy as np
import os
import re

import pytest

from paper_2206_02607_amd import crom

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "crom.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(crom_[a-z_0-9]+)\s*\(", text)))


def test_header_symbols_exported():
    L = crom.lib()
    names = _declared()
    assert len(names) >= 13
    for n in names:
        assert hasattr(L, n), n


def test_param_count_formula():
    # (m + r + 1) * w + (depth - 1) * (w + 1) * w + (w + 1) * d
    for m, r, d, w, depth in ((1, 3, 1, 32, 5), (2, 8, 1, 128, 5), (3, 16, 3, 256, 6)):
        expect = (m + r + 1) * w + (depth - 1) * (w + 1) * w + (w + 1) * d
        assert crom.param_count(m, r, d, w, depth) == expect
    assert crom.param_count(2, 8, 1, 128, 5) == 67585
    assert crom.param_count(3, 16, 3, 256, 6) == 334851


def _net(**kw):
    base = dict(m=2, r=8, d=1, width=128, depth=5, precision=1, act=0, _pad=0, params=1 << 20, packed=1 << 21)
    base.update(kw)
    return crom.CromNet(*[base[k] for k, _ in crom.CromNet._fields_])


def test_host_validation_before_launch():
    L = crom.lib()
    bad_shape = _net(width=96)
    assert L.crom_decode(ctypes.byref(bad_shape), 1, 10, 1, 1, None) == 2
    assert b"unsupported" in L.crom_last_error()
    assert L.crom_decode(None, 1, 10, 1, 1, None) == 1
    assert L.crom_decode(ctypes.byref(_net()), 1, -1, 1, 1, None) == 1
    assert L.crom_decode(ctypes.byref(_net()), None, 10, 1, 1, None) == 1
    assert L.crom_decode(ctypes.byref(_net(packed=None)), 1, 10, 1, 1, None) == 1
    assert L.crom_decode(ctypes.byref(_net(precision=7)), 1, 10, 1, 1, None) == 2
    # d2g given without a d2 mode, and the reverse
    assert L.crom_decode_jac(ctypes.byref(_net()), 1, 10, 1, 0, 1, None, 1, None, None) == 1
    assert L.crom_decode_jac(ctypes.byref(_net()), 1, 10, 1, 1, 1, None, None, None, None) == 1
    assert L.crom_decode_jac_q(ctypes.byref(_net()), 1, 10, 1, 1, None, None) == 1


def test_activation_validation():
    L = crom.lib()
    assert L.crom_decode(ctypes.byref(_net(act=2)), 1, 10, 1, 1, None) == 2
    assert b"activation" in L.crom_last_error()
    # sine: (1,3,1,32) and (2,8,1,128) in FP32 or BF16 only
    assert L.crom_decode(ctypes.byref(_net(act=1, precision=2)), 1, 10, 1, 1, None) == 2
    assert L.crom_decode(ctypes.byref(_net(act=1, m=3, r=16, d=3, width=256, depth=6)), 1, 10, 1, 1, None) == 2
    assert L.crom_decode(ctypes.byref(_net(act=1)), 1, 0, 1, 1, None) == 0  # P = 0: accepted, nothing to do
    n = ctypes.c_size_t(0)
    enc = crom.CromEncoder(16384, 256, 8, 0, 1 << 22)
    assert L.crom_train_workspace(ctypes.byref(_net(act=1, precision=0)), ctypes.byref(enc), 16, ctypes.byref(n)) == 2
    assert b"ELU" in L.crom_last_error()
    assert L.crom_train_workspace(ctypes.byref(_net(act=1)), ctypes.byref(enc), 16, ctypes.byref(n)) == 0
    assert L.crom_sampling_residual(ctypes.byref(_net(act=1)), 1 << 20, 10, 1, 1, 1, 1, 1, None, None) == 2


def test_step_validation():
    L = crom.lib()
    n = ctypes.c_size_t(0)
    assert L.crom_step_workspace(ctypes.byref(_net()), 4, 1000, ctypes.byref(n)) == 0
    assert n.value > 1000 * 8
    pde = crom.CromPDE(0, 0, 1e-4, 1 << 22)
    opts = crom.GNOptions().c_struct()
    args = dict(offsets=1 << 23, total=1000, y=1 << 24, clamp=None, qn=1 << 25, qnext=1 << 26,
                info=1 << 27, ws=1 << 28, wsb=n.value)

    def call(net=None, pde_=pde, opts_=opts, **kw):
        a = dict(args)
        a.update(kw)
        return L.crom_step(ctypes.byref(net or _net()), ctypes.byref(pde_), 4, a["offsets"], a["total"],
                           a["y"], a["clamp"], None, a["qn"], a["qnext"], ctypes.byref(opts_), a["info"],
                           a["ws"], a["wsb"], None)

    assert call(wsb=n.value - 1) == 3
    assert call(ws=(1 << 28) + 8) == 3                     # misaligned workspace
    assert call(qnext=1 << 25) == 1                        # aliasing q_n
    assert call(net=_net(m=3, r=16, d=3, width=256, depth=6)) == 2   # heat needs d == 1
    bad = crom.GNOptions(ls_shrink=1.5).c_struct()
    assert call(opts_=bad) == 1
    assert call(pde_=crom.CromPDE(0, 0, -1.0, 1 << 22)) == 1
    assert call(pde_=crom.CromPDE(5, 0, 1e-4, 1 << 22)) == 2
    assert call(pde_=crom.CromPDE(1, 0, 1e-4, 1 << 22)) == 2  # neo-Hookean needs m == d == 3
    assert call(pde_=crom.CromPDE(2, 0, 1e-4, 1 << 22)) == 2  # so does the FE step
    # the initial-guess variant: q_init must not alias q_next
    assert L.crom_step_guess(ctypes.byref(_net()), ctypes.byref(pde), 4, args["offsets"], args["total"], args["y"],
                             None, None, args["qn"], args["qnext"], args["qnext"], ctypes.byref(opts), args["info"],
                             args["ws"], args["wsb"], None) == 1


def test_fe_step_validation():
    L = crom.lib()
    net = _net(m=3, r=16, d=3, width=256, depth=6)
    n = ctypes.c_size_t(0)
    assert L.crom_step_workspace(ctypes.byref(net), 1, 500, ctypes.byref(n)) == 0
    opts = crom.GNOptions().c_struct()

    def call(mesh):
        pde = crom.CromPDE(2, 0, 1e-3, 1 << 22, None if mesh is None else ctypes.addressof(mesh))
        return L.crom_step(ctypes.byref(net), ctypes.byref(pde), 1, 1 << 23, 500, 1 << 24, None, None, 1 << 25,
                           1 << 26, ctypes.byref(opts), 1 << 27, 1 << 28, n.value, None)

    def mesh(**kw):
        f = dict(n_ring=6000, max_ring=6000, n_inc=10000, ring_offsets=1 << 29, ring_X=1 << 30, inc_offsets=1 << 31,
                 inc_tets=1 << 32, inc_corner=1 << 33, ring_u=1 << 34)
        f.update(kw)
        return crom.CromFEMesh(**f)

    assert call(None) == 1                        # the FE step needs its stencil
    assert call(mesh(max_ring=6001)) == 1         # larger than the whole ring
    assert call(mesh(n_inc=-1)) == 1
    assert call(mesh(ring_u=None)) == 1
    assert call(mesh(inc_corner=None)) == 1
    assert call(mesh(ring_offsets=None)) == 1


def test_heat_guess_and_encoder_validation():
    L = crom.lib()
    net = _net()  # (2, 8, 1, 128)
    n = ctypes.c_size_t(0)
    enc = crom.CromEncoder(16384, 256, 8, 0, 1 << 20)
    assert L.crom_heat_guess_workspace(ctypes.byref(net), ctypes.byref(enc), 2, 16384, ctypes.byref(n)) == 0
    assert n.value > 3 * 2 * 16384 * 4
    assert L.crom_heat_guess_workspace(ctypes.byref(net), ctypes.byref(enc), 2, 1000, ctypes.byref(n)) == 1
    assert L.crom_heat_guess_workspace(ctypes.byref(net), ctypes.byref(enc), 0, 16384, ctypes.byref(n)) == 1
    bad_r = crom.CromEncoder(16384, 256, 4, 0, 1 << 20)
    assert L.crom_heat_guess_workspace(ctypes.byref(net), ctypes.byref(bad_r), 2, 16384, ctypes.byref(n)) == 1
    net3 = _net(m=3, r=16, d=3, width=256, depth=6)
    enc3 = crom.CromEncoder(3 * 100, 32, 16, 0, 1 << 20)
    assert L.crom_heat_guess_workspace(ctypes.byref(net3), ctypes.byref(enc3), 1, 100, ctypes.byref(n)) == 2
    assert L.crom_heat_guess_workspace(ctypes.byref(net), ctypes.byref(enc), 2, 16384, ctypes.byref(n)) == 0
    assert L.crom_heat_guess(ctypes.byref(net), ctypes.byref(enc), 1 << 21, 16384, 2, 1 << 22, 1 << 23, 1e-4,
                             1 << 24, 1 << 25, n.value - 1, None) == 3
    # encoder kinds: the paper's convolutional encoder for 16,384 points
    # (four convolutions of 7 parameters, dense 63 -> 32, 32 -> 8)
    assert L.crom_conv_encoder_param_count(16384, 1, 32, 8) == 4 * 7 + 32 * 63 + 32 + 8 * 32 + 8
    assert L.crom_conv_encoder_param_count(40, 1, 32, 8) == 0   # no room for a convolution
    for kind, n_in, want in ((7, 16384, 1), (1, 40, 1), (1, 16384, 0)):
        e = crom.CromEncoder(n_in, 32, 8, kind, 1 << 20)
        assert L.crom_train_workspace(ctypes.byref(net), ctypes.byref(e), 4, ctypes.byref(n)) == want, (kind, n_in)


def test_sampling_validation():
    L = crom.lib()
    net = _net()  # (2, 8, 1, 128): r = 8, d = 1
    n = ctypes.c_size_t(0)

    def ws_query(n_try=10, max_samples=64, n_steps=500, kind=0, n_mu=40, P=16384):
        o = crom.CromSamplingOpts(n_try, max_samples, n_steps, 0.1)
        return L.crom_sampling_workspace(ctypes.byref(net), kind, n_mu, P, ctypes.byref(o), ctypes.byref(n))

    assert ws_query() == 0 and n.value > 11 * 16384 * 8
    assert ws_query(n_try=0) == 1
    assert ws_query(n_try=crom.SAMPLING_MAX_TRY + 1) == 1
    assert ws_query(max_samples=16385) == 1
    assert ws_query(n_steps=0) == 1
    assert ws_query(kind=7) == 1
    assert ws_query(n_mu=0) == 1
    assert ws_query() == 0
    wsb = n.value
    pde = crom.CromPDE(0, 0, 1e-4, 1 << 22)
    gn = crom.GNOptions().c_struct()
    o = crom.CromSamplingOpts(10, 64, 500, 0.1)
    res = crom.CromSamplingResult()

    def call(init, ws=1 << 28, wsb_=wsb, pde_=pde):
        s = np.zeros(64, dtype=np.int32)
        s[:len(init)] = init
        return L.crom_robust_sampling(ctypes.byref(net), ctypes.byref(pde_), 40, 1 << 21, 16384, None, 1 << 23,
                                      1 << 24, ctypes.byref(gn), ctypes.byref(o), s.ctypes.data_as(ctypes.c_void_p),
                                      len(init), ctypes.byref(res), None, None, ws, wsb_, None)

    good = list(range(0, 160, 10))
    assert call(good[:7]) == 1                     # r = 8 needs 8 samples
    assert call(good[:7] + [good[0]]) == 1        # repeated node
    assert call(good[:7] + [16384]) == 1          # node out of range
    assert call(good, wsb_=wsb - 1) == 3
    assert call(good, ws=(1 << 28) + 8) == 3
    assert call(good, pde_=crom.CromPDE(0, 0, 1e-4, None)) == 1
    assert L.crom_sampling_candidates(1 << 20, 100, None, 0, 1 << 21, None) == 1
    assert L.crom_sampling_candidates(1 << 20, 100, None, crom.SAMPLING_MAX_TRY + 1, 1 << 21, None) == 1
    assert L.crom_sampling_residual(ctypes.byref(net), 1 << 20, 0, 1, 1, 1, 1, 1, None, None) == 1
    assert L.crom_sampling_residual(ctypes.byref(net), 1 << 20, 10, 0, 1, 1, 1, 1, None, None) == 1
    assert L.crom_sampling_residual(ctypes.byref(net), 1 << 20, 10, 1, 1, 1, 1, None, None, None) == 1


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(crom, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(crom, "_lib", None)
    with pytest.raises(crom.CromError):
        crom.lib()
