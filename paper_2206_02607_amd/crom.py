"""Python binding of libcrom.so (include/crom.h): argument marshalling only.

Every computation runs in the library's HIP kernels; this module converts
torch tensors into device pointers and sizes, passes the current HIP stream
and raises on error codes.  It never falls back to another implementation:
if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, Structure, c_double, c_int32, c_int64, c_size_t, c_void_p
from dataclasses import dataclass
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# CROM_LIBRARY selects another build of the same library (the host
# sanitizer build); the default is the in-tree libcrom.so
LIB_PATH = os.environ.get("CROM_LIBRARY") or os.path.join(_HERE, "libcrom.so")

PREC_FP32, PREC_BF16, PREC_BF16_PURE, PREC_BF16X3 = 0, 1, 2, 3
D2_NONE, D2_LAPLACIAN, D2_HESSIAN = 0, 1, 2
PDE_HEAT, PDE_NEOHOOKEAN, PDE_COROTATED_FE, PDE_PROJECT = 0, 1, 2, 3
ACT_ELU, ACT_SINE = 0, 1
_ACT_NAMES = {"elu": ACT_ELU, "sine": ACT_SINE}
FLAG_MAXITER, FLAG_SINGULAR, FLAG_NONFINITE, FLAG_LS_FAIL, FLAG_ABORTED, FLAG_INVERTED = 1, 2, 4, 8, 16, 32
# a failed step: the rollout may hand the instance to the full-order fallback
FLAGS_FAILED = FLAG_SINGULAR | FLAG_NONFINITE | FLAG_LS_FAIL
_PREC_NAMES = {"fp32": PREC_FP32, "bf16": PREC_BF16, "bf16pure": PREC_BF16_PURE, "bf16x3": PREC_BF16X3}


class CromNet(Structure):
    _fields_ = [("m", c_int32), ("r", c_int32), ("d", c_int32), ("width", c_int32),
                ("depth", c_int32), ("precision", c_int32), ("act", c_int32), ("_pad", c_int32),
                ("params", c_void_p), ("packed", c_void_p)]


class CromPDE(Structure):
    _fields_ = [("kind", c_int32), ("_pad", c_int32), ("dt", c_double), ("coef", c_void_p), ("mesh", c_void_p)]


class CromFEMesh(Structure):
    _fields_ = [("n_ring", c_int64), ("max_ring", c_int64), ("n_inc", c_int64), ("ring_offsets", c_void_p),
                ("ring_X", c_void_p), ("inc_offsets", c_void_p), ("inc_tets", c_void_p),
                ("inc_corner", c_void_p), ("ring_u", c_void_p)]


class CromGNOpts(Structure):
    _fields_ = [("max_iter", c_int32), ("linearized", c_int32), ("ls_max", c_int32),
                ("max_rounds", c_int32), ("tol_step", c_double), ("armijo_c", c_double),
                ("ls_shrink", c_double)]


class CromEncoder(Structure):
    _fields_ = [("n_in", c_int32), ("hidden", c_int32), ("r", c_int32), ("kind", c_int32),
                ("params", c_void_p)]


class CromTrainStateLayout(Structure):
    _fields_ = [(n, c_size_t) for n in ("dec_params", "dec_grad", "dec_m", "dec_v", "enc_params", "enc_grad",
                                        "enc_m", "enc_v", "total")]


class CromSamplingOpts(Structure):
    _fields_ = [("n_try", c_int32), ("max_samples", c_int32), ("n_steps", c_int64), ("target", c_double)]


class CromSamplingResult(Structure):
    _fields_ = [("n_samples", c_int32), ("reached", c_int32), ("rounds", c_int32), ("_pad", c_int32),
                ("metric", c_double)]


INFO_DTYPE = np.dtype([("flags", "<i4"), ("iters", "<i4"), ("ls_evals", "<i4"), ("rounds", "<i4"),
                       ("obj_first", "<f8"), ("obj_last", "<f8")])

_lib = None


class CromError(RuntimeError):
    pass


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise CromError(f"{LIB_PATH} is missing: build it with "
                            "`python -m paper_2206_02607_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        L.crom_last_error.restype = ctypes.c_char_p
        L.crom_net_param_count.restype = c_size_t
        L.crom_net_param_count.argtypes = [c_int32] * 5
        L.crom_net_packed_bytes.restype = c_size_t
        L.crom_net_packed_bytes.argtypes = [POINTER(CromNet)]
        L.crom_net_pack.argtypes = [POINTER(CromNet), c_void_p, c_void_p]
        L.crom_decode.argtypes = [POINTER(CromNet), c_void_p, c_int64, c_void_p, c_void_p, c_void_p]
        L.crom_decode_jac.argtypes = [POINTER(CromNet), c_void_p, c_int64, c_void_p, c_int32,
                                      c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
        L.crom_decode_jac_x.argtypes = [POINTER(CromNet), c_void_p, c_int64, c_void_p, c_int32,
                                        c_void_p, c_void_p, c_void_p, c_void_p]
        L.crom_decode_jac_q.argtypes = [POINTER(CromNet), c_void_p, c_int64, c_void_p,
                                        c_void_p, c_void_p, c_void_p]
        L.crom_step_workspace.argtypes = [POINTER(CromNet), c_int32, c_int64, POINTER(c_size_t)]
        L.crom_step_targets.restype = c_void_p
        L.crom_step_targets.argtypes = [POINTER(CromNet), c_int32, c_int64, c_void_p]
        L.crom_step_increments.restype = c_void_p
        L.crom_step_increments.argtypes = [POINTER(CromNet), c_int32, c_int64, c_void_p]
        L.crom_step.argtypes = [POINTER(CromNet), POINTER(CromPDE), c_int32, c_void_p, c_int64,
                                c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, POINTER(CromGNOpts),
                                c_void_p, c_void_p, c_size_t, c_void_p]
        L.crom_fd_heat.argtypes = [c_int32, POINTER(c_int64), c_int64, c_void_p, c_int32, c_double,
                                   c_double, c_int64, c_void_p, c_void_p, c_void_p]
        L.crom_encoder_param_count.restype = c_size_t
        L.crom_encoder_param_count.argtypes = [c_int32] * 3
        L.crom_train_workspace.argtypes = [POINTER(CromNet), POINTER(CromEncoder), c_int32,
                                           POINTER(c_size_t)]
        L.crom_train_grads.argtypes = [POINTER(CromNet), POINTER(CromEncoder), c_void_p, c_void_p,
                                       c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                       c_size_t, c_void_p]
        L.crom_adam_step.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_int64,
                                     ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                     c_void_p]
        L.crom_train_step.argtypes = [POINTER(CromNet), c_void_p, c_void_p, c_void_p, c_void_p,
                                      POINTER(CromEncoder), c_void_p, c_void_p, c_void_p, c_int64,
                                      c_void_p, c_void_p, c_int32, ctypes.c_float, c_void_p,
                                      c_void_p, c_size_t, c_void_p]
        L.crom_encode_workspace.argtypes = [POINTER(CromNet), POINTER(CromEncoder), c_int32,
                                            POINTER(c_size_t)]
        L.crom_encode.argtypes = [POINTER(CromNet), POINTER(CromEncoder), c_void_p, c_int32, c_void_p,
                                  c_void_p, c_size_t, c_void_p]
        L.crom_decode_vjp_workspace.argtypes = [POINTER(CromNet), c_int32, c_int64, POINTER(c_size_t)]
        L.crom_decode_vjp.argtypes = [POINTER(CromNet), c_void_p, c_int64, c_void_p, c_int32,
                                      c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
        L.crom_sampling_residual.argtypes = [POINTER(CromNet), c_void_p, c_int64, c_int32, c_int32, c_void_p,
                                             c_void_p, c_void_p, c_void_p, c_void_p]
        L.crom_sampling_candidates.argtypes = [c_void_p, c_int64, c_void_p, c_int32, c_void_p, c_void_p]
        L.crom_sampling_workspace.argtypes = [POINTER(CromNet), c_int32, c_int32, c_int64,
                                              POINTER(CromSamplingOpts), POINTER(c_size_t)]
        L.crom_robust_sampling.argtypes = [POINTER(CromNet), POINTER(CromPDE), c_int32, c_void_p, c_int64,
                                           c_void_p, c_void_p, c_void_p, POINTER(CromGNOpts),
                                           POINTER(CromSamplingOpts), c_void_p, c_int32,
                                           POINTER(CromSamplingResult), c_void_p, c_void_p, c_void_p, c_size_t,
                                           c_void_p]
        L.crom_fe_stencil.argtypes = [c_int64, c_int64, c_void_p, c_int32, c_void_p, c_void_p,
                                      POINTER(c_int64), POINTER(c_int64), POINTER(c_int64), c_void_p,
                                      c_void_p, c_void_p, c_void_p, c_void_p]
        L.crom_conv_encoder_param_count.restype = c_size_t
        L.crom_conv_encoder_param_count.argtypes = [c_int64, c_int32, c_int32, c_int32]
        L.crom_step_guess.argtypes = [POINTER(CromNet), POINTER(CromPDE), c_int32, c_void_p, c_int64,
                                      c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                      POINTER(CromGNOpts), c_void_p, c_void_p, c_size_t, c_void_p]
        L.crom_heat_guess_workspace.argtypes = [POINTER(CromNet), POINTER(CromEncoder), c_int32, c_int64,
                                                POINTER(c_size_t)]
        L.crom_heat_guess.argtypes = [POINTER(CromNet), POINTER(CromEncoder), c_void_p, c_int64, c_int32,
                                      c_void_p, c_void_p, c_double, c_void_p, c_void_p, c_size_t, c_void_p]
        L.crom_standardization_of.argtypes = [c_void_p, c_int64, c_void_p, c_int64, c_int32, c_void_p, c_void_p]
        L.crom_standardize.argtypes = [c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_int64, c_int32,
                                       c_void_p, c_void_p]
        L.crom_fold_standardization.argtypes = [POINTER(CromNet), POINTER(CromEncoder), c_void_p, c_void_p]
        L.crom_train_state_offsets.argtypes = [POINTER(CromNet), POINTER(CromEncoder), c_void_p]
        L.crom_train_state_bytes.restype = c_size_t
        L.crom_train_state_bytes.argtypes = [POINTER(CromNet), POINTER(CromEncoder)]
        L.crom_train_step_state.argtypes = [POINTER(CromNet), POINTER(CromEncoder), c_void_p, c_void_p, c_int64,
                                            c_void_p, c_void_p, c_int32, ctypes.c_float, c_void_p, c_void_p,
                                            c_size_t, c_void_p]
        L.crom_step_static_capacity.restype = c_size_t
        L.crom_step_static_capacity.argtypes = []
        L.crom_step_static.argtypes = [POINTER(CromNet), POINTER(CromPDE), c_int32, c_void_p, c_int64, c_void_p,
                                       c_void_p, c_void_p, c_void_p, c_void_p, POINTER(CromGNOpts), c_void_p,
                                       c_void_p]
        L.crom_heat_fallback_workspace.argtypes = [POINTER(CromNet), c_int32, c_int64, c_int64, POINTER(c_size_t)]
        L.crom_heat_fallback.argtypes = [POINTER(CromNet), c_void_p, c_int64, c_int64, c_double, c_int32, c_int32,
                                         c_void_p, c_void_p, c_void_p, c_double, c_int64, POINTER(CromGNOpts),
                                         c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
        L.crom_kernel_timer.argtypes = [c_int32]
        L.crom_kernel_timer_read.argtypes = [POINTER(c_double), POINTER(c_int64)]
        for name in ("crom_sampling_residual", "crom_sampling_candidates", "crom_sampling_workspace",
                     "crom_robust_sampling", "crom_kernel_timer", "crom_kernel_timer_read", "crom_fe_stencil", "crom_step_guess", "crom_heat_guess_workspace",
                     "crom_heat_guess", "crom_standardization_of", "crom_standardize",
                     "crom_fold_standardization", "crom_train_state_offsets", "crom_train_step_state",
                     "crom_step_static", "crom_heat_fallback_workspace", "crom_heat_fallback"):
            getattr(L, name).restype = c_int32
        for name in ("crom_net_pack", "crom_decode", "crom_decode_jac", "crom_decode_jac_x",
                     "crom_decode_jac_q", "crom_step_workspace", "crom_step", "crom_fd_heat",
                     "crom_train_workspace", "crom_train_grads", "crom_adam_step", "crom_train_step",
                     "crom_decode_vjp_workspace", "crom_decode_vjp", "crom_encode_workspace",
                     "crom_encode"):
            getattr(L, name).restype = c_int32
        _lib = L
    return _lib


def _check(status: int, what: str) -> None:
    if status != 0:
        raise CromError(f"{what} failed ({status}): {lib().crom_last_error().decode()}")


def _torch():
    import torch
    return torch


def _stream() -> c_void_p:
    torch = _torch()
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise CromError("device tensor expected")
    if not t.is_contiguous():
        raise CromError("contiguous tensor expected")
    return t.data_ptr()


def param_count(m: int, r: int, d: int, width: int, depth: int) -> int:
    return int(lib().crom_net_param_count(m, r, d, width, depth))


def flatten_layers(layers: Sequence[Tuple[np.ndarray, np.ndarray]]) -> np.ndarray:
    """Natural parameter layout: W_1, b_1, W_2, b_2, ... as one FP32 vector."""
    parts = []
    for W, b in layers:
        parts.append(np.asarray(W, dtype=np.float32).ravel())
        parts.append(np.asarray(b, dtype=np.float32).ravel())
    return np.concatenate(parts)


class Decoder:
    """A decoder g(x, q) resident on the GPU: FP32 parameters plus the packed
    fragment copy for the chosen precision."""

    def __init__(self, params, m: int, r: int, d: int, width: int, depth: int,
                 precision="bf16", device="cuda", act="elu"):
        torch = _torch()
        self.m, self.r, self.d, self.width, self.depth = m, r, d, width, depth
        self.precision = _PREC_NAMES[precision] if isinstance(precision, str) else int(precision)
        self.act = _ACT_NAMES[act] if isinstance(act, str) else int(act)
        n = param_count(m, r, d, width, depth)
        if isinstance(params, np.ndarray):
            params = torch.from_numpy(np.ascontiguousarray(params, dtype=np.float32))
        params = params.to(device=device, dtype=torch.float32).contiguous()
        if params.numel() != n:
            raise CromError(f"expected {n} parameters, got {params.numel()}")
        self.params = params
        nb = int(lib().crom_net_packed_bytes(ctypes.byref(self._net(packed=False))))
        self.packed = torch.empty(max(nb, 256), dtype=torch.uint8, device=device)
        self.pack()

    @classmethod
    def from_layers(cls, layers, m: int, precision="bf16", device="cuda", act="elu"):
        r = layers[0][0].shape[1] - m
        return cls(flatten_layers(layers), m, r, layers[-1][0].shape[0], layers[0][0].shape[0],
                   len(layers) - 1, precision, device, act)

    def _net(self, packed=True) -> CromNet:
        return CromNet(self.m, self.r, self.d, self.width, self.depth, self.precision, self.act, 0,
                       self.params.data_ptr(), self.packed.data_ptr() if packed else None)

    def pack(self) -> None:
        net = self._net(packed=False)
        _check(lib().crom_net_pack(ctypes.byref(net), self.packed.data_ptr(), _stream()), "crom_net_pack")

    # -- decode ---------------------------------------------------------
    def _prep(self, x, q):
        torch = _torch()
        x = x.to(dtype=torch.float32).contiguous()
        q = q.to(device=x.device, dtype=torch.float64).contiguous()
        if x.dim() != 2 or x.shape[1] != self.m or q.numel() != self.r:
            raise CromError("x must be [P, m] and q [r]")
        return x, q

    def decode(self, x, q, out=None):
        torch = _torch()
        x, q = self._prep(x, q)
        P = x.shape[0]
        g = out if out is not None else torch.empty(P, self.d, dtype=torch.float32, device=x.device)
        net = self._net()
        _check(lib().crom_decode(ctypes.byref(net), _ptr(x), P, _ptr(q), _ptr(g), _stream()), "crom_decode")
        return g

    def decode_jac(self, x, q, dx=True, d2=D2_NONE, dq=True):
        """Returns (g, dgdx | None, d2g | None, dgdq | None)."""
        torch = _torch()
        x, q = self._prep(x, q)
        P, dev = x.shape[0], x.device
        f32 = dict(dtype=torch.float32, device=dev)
        g = torch.empty(P, self.d, **f32)
        gx = torch.empty(P, self.d, self.m, **f32) if dx else None
        if d2 == D2_LAPLACIAN:
            h = torch.empty(P, self.d, **f32)
        elif d2 == D2_HESSIAN:
            h = torch.empty(P, self.d, self.m * (self.m + 1) // 2, **f32)
        else:
            h = None
        gq = torch.empty(P, self.d, self.r, **f32) if dq else None
        net = self._net()
        _check(lib().crom_decode_jac(ctypes.byref(net), _ptr(x), P, _ptr(q), int(d2), _ptr(g),
                                     _ptr(gx), _ptr(h), _ptr(gq), _stream()), "crom_decode_jac")
        return g, gx, h, gq

    def decode_jac_x(self, x, q, d2=D2_LAPLACIAN):
        torch = _torch()
        x, q = self._prep(x, q)
        P, dev = x.shape[0], x.device
        f32 = dict(dtype=torch.float32, device=dev)
        g = torch.empty(P, self.d, **f32)
        gx = torch.empty(P, self.d, self.m, **f32)
        nh = {D2_NONE: 0, D2_LAPLACIAN: 1, D2_HESSIAN: self.m * (self.m + 1) // 2}[d2]
        h = torch.empty(P, self.d, nh, **f32).squeeze(-1) if nh else None
        net = self._net()
        _check(lib().crom_decode_jac_x(ctypes.byref(net), _ptr(x), P, _ptr(q), int(d2), _ptr(g),
                                       _ptr(gx), _ptr(h), _stream()), "crom_decode_jac_x")
        return g, gx, h

    def decode_jac_q(self, x, q):
        torch = _torch()
        x, q = self._prep(x, q)
        P, dev = x.shape[0], x.device
        g = torch.empty(P, self.d, dtype=torch.float32, device=dev)
        gq = torch.empty(P, self.d, self.r, dtype=torch.float32, device=dev)
        net = self._net()
        _check(lib().crom_decode_jac_q(ctypes.byref(net), _ptr(x), P, _ptr(q), _ptr(g), _ptr(gq),
                                       _stream()), "crom_decode_jac_q")
        return g, gq


def decode_vjp(dec: "Decoder", x, q, dg):
    """Backward of the decoder over B latents: q [B, r] FP32, dg [B, P, d]
    cotangent of g(x_p, q_b).  Returns (grad_params [n_params], grad_q [B, r])."""
    torch = _torch()
    x = x.to(dtype=torch.float32).contiguous()
    q = q.to(device=x.device, dtype=torch.float32).contiguous()
    dg = dg.to(device=x.device, dtype=torch.float32).contiguous()
    B, P = q.shape[0], x.shape[0]
    if q.dim() != 2 or q.shape[1] != dec.r or dg.numel() != B * P * dec.d:
        raise CromError("q must be [B, r] and dg [B, P, d]")
    net = dec._net(packed=False)
    nbytes = c_size_t(0)
    _check(lib().crom_decode_vjp_workspace(ctypes.byref(net), B, P, ctypes.byref(nbytes)),
           "crom_decode_vjp_workspace")
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=x.device)
    gp = torch.empty_like(dec.params)
    gq = torch.empty(B, dec.r, dtype=torch.float32, device=x.device)
    _check(lib().crom_decode_vjp(ctypes.byref(net), _ptr(x), P, _ptr(q), B, _ptr(dg), _ptr(gp),
                                 _ptr(gq), _ptr(ws), nbytes.value, _stream()), "crom_decode_vjp")
    return gp, gq


ENC_DENSE, ENC_CONV = 0, 1
_ENC_NAMES = {"dense": ENC_DENSE, "conv": ENC_CONV}


def encoder_param_count(n_in: int, hidden: int, r: int, kind: str = "dense", d: int = 1) -> int:
    """FP32 parameters of an encoder: dense (n_in inputs) or convolutional
    (n_in = P d values of P points with d channels)."""
    if kind == "conv":
        return int(lib().crom_conv_encoder_param_count(n_in // d, d, hidden, r))
    return int(lib().crom_encoder_param_count(n_in, hidden, r))


class Trainer:
    """Encoder + decoder training on the GPU (crom_train_grads / crom_train_step).

    dec: the Decoder whose FP32 params are the master copy (updated in place,
    packed weights refreshed after every step); enc_params: the encoder's FP32
    parameters in the layout of its kind (dense [E1, c1, E2, c2]; "conv" the
    convolutions' [W, b] then [E1, c1, E2, c2]; updated in place); x [P, m]
    the snapshot points; B the batch size."""

    def __init__(self, dec: "Decoder", enc_params, hidden: int, x, B: int, enc_kind: str = "dense"):
        torch = _torch()
        self.dec, self.hidden, self.B = dec, hidden, B
        self.x = x.to(dtype=torch.float32).contiguous()
        self.P = self.x.shape[0]
        self.n_in = self.P * dec.d
        self.enc_kind = _ENC_NAMES[enc_kind]
        ne = encoder_param_count(self.n_in, hidden, dec.r, enc_kind, dec.d)
        if isinstance(enc_params, np.ndarray):
            enc_params = torch.from_numpy(np.ascontiguousarray(enc_params, dtype=np.float32))
        self.enc_params = enc_params.to(device=self.x.device, dtype=torch.float32).contiguous()
        if self.enc_params.numel() != ne:
            raise CromError(f"expected {ne} encoder parameters, got {self.enc_params.numel()}")
        dev = self.x.device
        nbytes = c_size_t(0)
        _check(lib().crom_train_workspace(ctypes.byref(dec._net(packed=False)), ctypes.byref(self._enc()),
                                          B, ctypes.byref(nbytes)), "crom_train_workspace")
        self.ws = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
        # the training state blob (crom_train_state_offsets): the decoder's
        # and encoder's parameters, gradients and Adam moments; the Decoder
        # and this trainer hold views into it
        lay = CromTrainStateLayout()
        _check(lib().crom_train_state_offsets(ctypes.byref(dec._net(packed=False)), ctypes.byref(self._enc()),
                                              ctypes.byref(lay)), "crom_train_state_offsets")
        self.layout = lay
        self._state_raw = torch.zeros(lay.total + 256, dtype=torch.uint8, device=dev)
        a0 = (256 - self._state_raw.data_ptr() % 256) % 256
        self.state = self._state_raw[a0:a0 + lay.total]
        nd = dec.params.numel()

        def view(off, n):
            return self.state[off:off + 4 * n].view(torch.float32)

        view(lay.dec_params, nd).copy_(dec.params)
        view(lay.enc_params, ne).copy_(self.enc_params)
        dec.params = view(lay.dec_params, nd)
        self.enc_params = view(lay.enc_params, ne)
        self.grad_dec, self.m_dec, self.v_dec = view(lay.dec_grad, nd), view(lay.dec_m, nd), view(lay.dec_v, nd)
        self.grad_enc, self.m_enc, self.v_enc = view(lay.enc_grad, ne), view(lay.enc_m, ne), view(lay.enc_v, ne)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.q = torch.zeros(B, dec.r, dtype=torch.float32, device=dev)
        self.t = 0

    def _enc(self) -> CromEncoder:
        return CromEncoder(self.n_in, self.hidden, self.dec.r, self.enc_kind, self.enc_params.data_ptr())

    def _u(self, u):
        torch = _torch()
        u = u.to(device=self.x.device, dtype=torch.float32).contiguous()
        if u.numel() != self.B * self.n_in:
            raise CromError(f"u must hold B x P x d = {self.B * self.n_in} values")
        return u

    def grads(self, u):
        """Loss and gradients of one batch u [B, P(, d)] without an update.
        Returns (loss [1], grad_dec, grad_enc, q [B, r]) (views of internal buffers)."""
        u = self._u(u)
        net, enc = self.dec._net(packed=False), self._enc()
        _check(lib().crom_train_grads(ctypes.byref(net), ctypes.byref(enc), _ptr(u), _ptr(self.x),
                                      self.B, _ptr(self.grad_dec), _ptr(self.grad_enc), _ptr(self.loss),
                                      _ptr(self.q), _ptr(self.ws), self.ws.numel(), _stream()),
               "crom_train_grads")
        return self.loss, self.grad_dec, self.grad_enc, self.q

    def step(self, u, lr: float = 1e-3):
        """One Adam step on batch u; returns the batch loss (device tensor [1])
        measured before the update."""
        u = self._u(u)
        self.t += 1
        net, enc = self.dec._net(packed=False), self._enc()
        _check(lib().crom_train_step_state(ctypes.byref(net), ctypes.byref(enc), _ptr(self.state),
                                           _ptr(self.dec.packed), self.t, _ptr(u), _ptr(self.x), self.B, lr,
                                           _ptr(self.loss), _ptr(self.ws), self.ws.numel(), _stream()),
               "crom_train_step_state")
        return self.loss

    def checkpoint(self):
        """(a copy of the state blob, the Adam step): everything a resumed
        run needs besides the data order."""
        return self.state.clone(), self.t

    def restore(self, ckpt) -> None:
        """Resume from a checkpoint (copies the blob in, re-packs the decoder)."""
        blob, t = ckpt
        if blob.numel() != self.state.numel():
            raise CromError("checkpoint of another layout")
        self.state.copy_(blob)
        self.t = int(t)
        self.dec.pack()

    def encode(self, u):
        """Latents q [n, r] FP32 of the snapshots u [n, P(, d)], any n >= 1
        (encoder forward only, crom_encode)."""
        torch = _torch()
        u = u.to(device=self.x.device, dtype=torch.float32).contiguous()
        n = u.numel() // self.n_in
        if n < 1 or u.numel() != n * self.n_in:
            raise CromError(f"u must hold n x {self.n_in} values")
        net, enc = self.dec._net(packed=False), self._enc()
        nbytes = c_size_t(0)
        _check(lib().crom_encode_workspace(ctypes.byref(net), ctypes.byref(enc), n, ctypes.byref(nbytes)),
               "crom_encode_workspace")
        ws = torch.empty(nbytes.value, dtype=torch.uint8, device=self.x.device)
        q = torch.empty(n, self.dec.r, dtype=torch.float32, device=self.x.device)
        _check(lib().crom_encode(ctypes.byref(net), ctypes.byref(enc), _ptr(u), n, _ptr(q), _ptr(ws),
                                 nbytes.value, _stream()), "crom_encode")
        return q


def heat_guess(dec: "Decoder", enc_params, hidden: int, nodes, q_n, nu, dt: float, enc_kind: str = "dense"):
    """Encoder-based initial guesses [n, r] FP64 for the heat step
    (crom_heat_guess): the encoder (FP32 params [E1, c1, E2, c2], n_in =
    P * d) applied to g + dt nu Laplacian g over all nodes [P, m] for each
    latent q_n [n, r]; nu one value or one per instance."""
    torch = _torch()
    dev = dec.params.device
    nodes = nodes.to(device=dev, dtype=torch.float32).contiguous()
    q_n = torch.as_tensor(q_n, dtype=torch.float64, device=dev).reshape(-1, dec.r).contiguous()
    n, P = q_n.shape[0], nodes.shape[0]
    nu = torch.as_tensor(nu, dtype=torch.float64, device=dev).reshape(-1).expand(n).contiguous()
    enc_params = torch.as_tensor(enc_params, dtype=torch.float32, device=dev).contiguous()
    enc = CromEncoder(P * dec.d, hidden, dec.r, _ENC_NAMES[enc_kind], enc_params.data_ptr())
    net = dec._net()
    nbytes = c_size_t(0)
    _check(lib().crom_heat_guess_workspace(ctypes.byref(net), ctypes.byref(enc), n, P, ctypes.byref(nbytes)),
           "crom_heat_guess_workspace")
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=dev)
    out = torch.empty(n, dec.r, dtype=torch.float64, device=dev)
    _check(lib().crom_heat_guess(ctypes.byref(net), ctypes.byref(enc), _ptr(nodes), P, n, _ptr(q_n), _ptr(nu),
                                 float(dt), _ptr(out), _ptr(ws), nbytes.value, _stream()), "crom_heat_guess")
    return out


# ---------------------------------------------------------------------------
# Standardization of the training data and its fold (Sec. "Training Details").
# A crom_standardization is 8 doubles on the device: u_mean, u_std,
# x_mean[3], x_std[3].
# ---------------------------------------------------------------------------
def standardization_of(u, x):
    """Moments of the FP64 snapshots u (every value) and of the FP32 nodes
    x [P, m]: a float64 device tensor of 8 values (crom_standardization)."""
    torch = _torch()
    u = u.to(dtype=torch.float64).contiguous()
    x = x.to(device=u.device, dtype=torch.float32).contiguous()
    s = torch.empty(8, dtype=torch.float64, device=u.device)
    _check(lib().crom_standardization_of(_ptr(u), u.numel(), _ptr(x), x.shape[0], x.shape[1], _ptr(s), _stream()),
           "crom_standardization_of")
    return s


def standardize(s, u=None, x=None):
    """(u_s, x_s) FP32 standardized copies of u (FP64, any shape) and x
    [P, m] (either may be None)."""
    torch = _torch()
    u_s = x_s = None
    n_u, P, m = 0, 0, 1
    if u is not None:
        u = u.to(dtype=torch.float64).contiguous()
        u_s = torch.empty(u.shape, dtype=torch.float32, device=u.device)
        n_u = u.numel()
    if x is not None:
        x = x.to(dtype=torch.float32).contiguous()
        x_s = torch.empty_like(x)
        P, m = x.shape
    _check(lib().crom_standardize(_ptr(s), _ptr(u), n_u, _ptr(u_s), _ptr(x), P, m, _ptr(x_s), _stream()),
           "crom_standardize")
    return u_s, x_s


def fold_standardization(dec: "Decoder", s, enc_params=None, n_in: int = 0, hidden: int = 0,
                         enc_kind: str = "dense") -> None:
    """Folds the standardization s into the decoder and, when enc_params is
    given (FP32 device params of an encoder of kind enc_kind with n_in = P d
    inputs), into the encoder, in place; then re-packs the decoder."""
    enc = None
    if enc_params is not None:
        if enc_params.dtype != _torch().float32 or not enc_params.is_cuda or not enc_params.is_contiguous():
            raise CromError("encoder params must be a contiguous FP32 device tensor")
        enc = CromEncoder(n_in, hidden, dec.r, _ENC_NAMES[enc_kind], enc_params.data_ptr())
    net = dec._net(packed=False)
    _check(lib().crom_fold_standardization(ctypes.byref(net), ctypes.byref(enc) if enc is not None else None,
                                           _ptr(s), _stream()), "crom_fold_standardization")
    dec.pack()


class HeatFallback:
    """The full-order fallback of failed heat steps (crom_heat_fallback):
    decode at the grid nodes [nx * ny, 2] (index i_x * ny + i_y), FP64
    finite-difference update with substep dt_fd, projection back onto the
    decoder at every node (Gauss-Newton with `opts`)."""

    def __init__(self, dec: "Decoder", nodes, nx: int, ny: int, dx: float, dt_fd: float,
                 opts: "GNOptions" = None):
        torch = _torch()
        self.dec, self.nx, self.ny, self.dx, self.dt_fd = dec, nx, ny, dx, dt_fd
        self.opts = opts if opts is not None else GNOptions(max_iter=3, tol_step=1e-6)
        self.nodes = nodes.to(device=dec.params.device, dtype=torch.float32).contiguous()
        self._ws = {}

    def __call__(self, failed, q_last, nu, dt: float, q_next, info_buf=None) -> None:
        """Replace q_next of the instances in `failed` (host ints) by the
        projected full-order update of their fields over dt from q_last."""
        torch = _torch()
        inst = (ctypes.c_int32 * len(failed))(*[int(i) for i in failed])
        n = len(failed)
        substeps = int(round(dt / self.dt_fd))
        if abs(substeps * self.dt_fd - dt) > 1e-9 * dt:
            raise CromError("dt must be a multiple of the finite-difference substep")
        net = self.dec._net()
        if n not in self._ws:
            nbytes = c_size_t(0)
            _check(lib().crom_heat_fallback_workspace(ctypes.byref(net), n, self.nx, self.ny, ctypes.byref(nbytes)),
                   "crom_heat_fallback_workspace")
            self._ws[n] = torch.empty(nbytes.value, dtype=torch.uint8, device=q_next.device)
        ws = self._ws[n]
        nu = torch.as_tensor(nu, dtype=torch.float64, device=q_next.device).reshape(-1).contiguous()
        self._nu = nu
        o = self.opts.c_struct()
        _check(lib().crom_heat_fallback(ctypes.byref(net), _ptr(self.nodes), self.nx, self.ny, self.dx,
                                        q_next.shape[0], n, inst, _ptr(q_last), _ptr(nu), self.dt_fd, substeps,
                                        ctypes.byref(o), _ptr(q_next),
                                        info_buf.data_ptr() if info_buf is not None else None, _ptr(ws),
                                        ws.numel(), _stream()), "crom_heat_fallback")


def adam_step(params, grad, m, v, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam update of FP32 device tensors."""
    _check(lib().crom_adam_step(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), params.numel(), t, lr,
                                beta1, beta2, eps, _stream()), "crom_adam_step")


@dataclass
class GNOptions:
    max_iter: int = 5
    linearized: bool = False
    ls_max: int = 10
    tol_step: float = 1e-6
    armijo_c: float = 1e-4
    ls_shrink: float = 0.5
    max_rounds: int = 0

    def c_struct(self) -> CromGNOpts:
        return CromGNOpts(self.max_iter, int(self.linearized), self.ls_max, self.max_rounds,
                          self.tol_step, self.armijo_c, self.ls_shrink)


class FEStencil:
    """Finite-element stencil of each instance's sample vertices on a
    tetrahedral mesh (crom_fe_stencil on the host), uploaded in the layout
    crom_fe_mesh takes.

    X [V, 3] rest positions, tets [T, 4] vertex indices, samples: one array
    of sample vertex indices per instance.  Attributes: offsets and y (the
    samples' CSR offsets and positions, for Stepper), ring_vert (mesh vertex
    of each ring entry, host), ring_u (the decoded ring displacement a step
    writes, device)."""

    def __init__(self, X, tets, samples: Sequence, device):
        torch = _torch()
        X = np.ascontiguousarray(np.asarray(X, dtype=np.float32))
        tets = np.ascontiguousarray(np.asarray(tets, dtype=np.int32))
        sv = [np.asarray(sm, dtype=np.int32) for sm in samples]
        soff = np.zeros(len(sv) + 1, dtype=np.int64)
        soff[1:] = np.cumsum([len(a) for a in sv])
        svert = np.ascontiguousarray(np.concatenate(sv) if sv else np.zeros(0, np.int32))
        n_ring, max_ring, n_inc = c_int64(0), c_int64(0), c_int64(0)
        args = (X.shape[0], tets.shape[0], tets.ctypes.data, len(sv), soff.ctypes.data, svert.ctypes.data,
                ctypes.byref(n_ring), ctypes.byref(max_ring), ctypes.byref(n_inc))
        _check(lib().crom_fe_stencil(*args, None, None, None, None, None), "crom_fe_stencil")
        ring_off = np.zeros(len(sv) + 1, dtype=np.int64)
        ring_vert = np.zeros(n_ring.value, dtype=np.int32)
        inc_off = np.zeros(int(soff[-1]) + 1, dtype=np.int64)
        inc_tets = np.zeros((n_inc.value, 4), dtype=np.int32)
        inc_corner = np.zeros(n_inc.value, dtype=np.int8)
        _check(lib().crom_fe_stencil(*args, ring_off.ctypes.data, ring_vert.ctypes.data, inc_off.ctypes.data,
                                     inc_tets.ctypes.data, inc_corner.ctypes.data), "crom_fe_stencil")
        self.n_ring, self.max_ring, self.n_inc = n_ring.value, max_ring.value, n_inc.value
        self.ring_vert = ring_vert
        self.sample_vert = svert
        to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
        self.offsets = to(soff)
        self.y = to(X[svert])
        self.ring_offsets = to(ring_off)
        self.ring_X = to(X[ring_vert])
        self.inc_offsets = to(inc_off)
        self.inc_tets = to(inc_tets)
        self.inc_corner = to(inc_corner)
        self.ring_u = torch.zeros(max(self.n_ring, 1), 3, dtype=torch.float32, device=device)

    def c_struct(self) -> CromFEMesh:
        return CromFEMesh(self.n_ring, self.max_ring, self.n_inc, _ptr(self.ring_offsets), _ptr(self.ring_X),
                          _ptr(self.inc_offsets), _ptr(self.inc_tets), _ptr(self.inc_corner), _ptr(self.ring_u))


class Stepper:
    """Reusable latent-step launcher for a fixed batch layout (instances,
    CSR sample offsets, sample points): owns the workspace.  pde "heat",
    "neohookean" or "corotated_fe" (then `mesh` is the FEStencil whose
    offsets and y these are)."""

    def __init__(self, dec: Decoder, offsets, y, clamp=None, pde: str = "heat", mesh: "FEStencil" = None):
        torch = _torch()
        self.dec = dec
        self.kind = {"heat": PDE_HEAT, "neohookean": PDE_NEOHOOKEAN, "corotated_fe": PDE_COROTATED_FE,
                     "project": PDE_PROJECT}[pde]
        if (self.kind == PDE_COROTATED_FE) != (mesh is not None):
            raise CromError("the finite-element step, and only it, takes a mesh stencil")
        self.mesh = mesh
        off = torch.as_tensor(offsets, dtype=torch.int64)
        self.n_inst = int(off.numel() - 1)
        self.total = int(off[-1].item())
        self.offsets = off.to(dec.params.device).contiguous()
        self.y = y.to(device=dec.params.device, dtype=torch.float32).contiguous()
        if self.y.shape != (self.total, dec.m):
            raise CromError("y must be [total_samples, m]")
        self.clamp = None if clamp is None else clamp.to(device=dec.params.device, dtype=torch.uint8).contiguous()
        nbytes = c_size_t(0)
        net = dec._net()
        _check(lib().crom_step_workspace(ctypes.byref(net), self.n_inst, self.total, ctypes.byref(nbytes)),
               "crom_step_workspace")
        self.ws = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=dec.params.device)
        base = self.ws.data_ptr()
        self.ws_ptr = (base + 255) // 256 * 256
        self.ws_bytes = int(nbytes.value)
        self.info_buf = torch.zeros(self.n_inst * INFO_DTYPE.itemsize, dtype=torch.uint8,
                                    device=dec.params.device)

    def step(self, q_n, coef, dt: float, opts: GNOptions = GNOptions(), q_next=None, q_prev=None, q_init=None):
        """One latent step.  coef: heat, nu (one value or one per instance);
        neo-Hookean and corotated, (lam, mu, rho0, Bx, By, Bz) (one row or one
        per instance).  q_prev: the elastic kinds, the previous latents (None:
        at rest).  q_init: a second candidate start per instance
        (crom_step_guess; None: crom_step)."""
        torch = _torch()
        dev = self.dec.params.device
        q_n = q_n.to(device=dev, dtype=torch.float64).contiguous()
        coef = self._coef_tensor(coef)
        if q_prev is not None:
            q_prev = q_prev.to(device=dev, dtype=torch.float64).contiguous()
        if q_next is None:
            q_next = torch.empty_like(q_n)
        net = self.dec._net()
        fm = self.mesh.c_struct() if self.mesh is not None else None
        pde = CromPDE(self.kind, 0, float(dt), coef.data_ptr(), ctypes.addressof(fm) if fm is not None else None)
        o = opts.c_struct()
        self._coef, self._q_prev = coef, q_prev  # keep alive until the stream has consumed them
        if q_init is None:
            _check(lib().crom_step(ctypes.byref(net), ctypes.byref(pde), self.n_inst, _ptr(self.offsets),
                                   self.total, _ptr(self.y), _ptr(self.clamp), _ptr(q_prev), _ptr(q_n),
                                   _ptr(q_next), ctypes.byref(o), self.info_buf.data_ptr(), self.ws_ptr,
                                   self.ws_bytes, _stream()), "crom_step")
            return q_next
        q_init = q_init.to(device=dev, dtype=torch.float64).contiguous()
        self._q_init = q_init
        _check(lib().crom_step_guess(ctypes.byref(net), ctypes.byref(pde), self.n_inst, _ptr(self.offsets),
                                     self.total, _ptr(self.y), _ptr(self.clamp), _ptr(q_prev), _ptr(q_n),
                                     _ptr(q_init), _ptr(q_next), ctypes.byref(o), self.info_buf.data_ptr(),
                                     self.ws_ptr, self.ws_bytes, _stream()), "crom_step_guess")
        return q_next

    def _coef_tensor(self, coef):
        """The per-instance coefficients as the library reads them (heat: nu;
        elastic kinds: 6 values; projection: the targets [total] FP64)."""
        torch = _torch()
        dev = self.dec.params.device
        if self.kind == PDE_PROJECT:
            coef = torch.as_tensor(coef, dtype=torch.float64, device=dev).reshape(-1).contiguous()
            if coef.numel() != self.total * self.dec.d:
                raise CromError("the projection takes one target per sample and output")
            return coef
        per = 1 if self.kind == PDE_HEAT else 6
        coef = torch.as_tensor(coef, dtype=torch.float64, device=dev).reshape(-1, per)
        return coef.expand(self.n_inst, per).contiguous()

    def step_static(self, q_n, coef, dt: float, opts: GNOptions = GNOptions(), q_next=None, q_prev=None):
        """crom_step_static: the same step with the library's own workspace
        (no allocation by the call; this object's workspace is not used)."""
        torch = _torch()
        dev = self.dec.params.device
        q_n = q_n.to(device=dev, dtype=torch.float64).contiguous()
        coef = self._coef_tensor(coef)
        if q_prev is not None:
            q_prev = q_prev.to(device=dev, dtype=torch.float64).contiguous()
        if q_next is None:
            q_next = torch.empty_like(q_n)
        net = self.dec._net()
        fm = self.mesh.c_struct() if self.mesh is not None else None
        pde = CromPDE(self.kind, 0, float(dt), coef.data_ptr(), ctypes.addressof(fm) if fm is not None else None)
        o = opts.c_struct()
        self._coef, self._q_prev = coef, q_prev
        _check(lib().crom_step_static(ctypes.byref(net), ctypes.byref(pde), self.n_inst, _ptr(self.offsets),
                                      self.total, _ptr(self.y), _ptr(self.clamp), _ptr(q_prev), _ptr(q_n),
                                      _ptr(q_next), ctypes.byref(o), self.info_buf.data_ptr(), _stream()),
               "crom_step_static")
        return q_next

    def info(self) -> np.ndarray:
        """Per-instance outcome of the last step (synchronises)."""
        return np.frombuffer(self.info_buf.cpu().numpy().tobytes(), dtype=INFO_DTYPE)

    def _ws_view(self, fn):
        torch = _torch()
        n = self.total * self.dec.d
        off = self.ws_ptr - self.ws.data_ptr()
        net = self.dec._net()
        p = fn(ctypes.byref(net), self.n_inst, self.total, c_void_p(self.ws_ptr))
        start = off + (p - self.ws_ptr)
        return self.ws[start:start + 8 * n].view(torch.float64).reshape(self.total, self.dec.d)

    def targets(self):
        """FP64 targets f_{n+1} [total, d] of the last step (a view into the workspace)."""
        return self._ws_view(lib().crom_step_targets)

    def increments(self):
        """FP64 increments rho_0 = f_{n+1} - g(q_n) [total, d] of the last step (a view)."""
        return self._ws_view(lib().crom_step_increments)


def fd_heat(u, nu, dx: float, dt: float, steps: int, scratch=None):
    """Full-order FP64 heat solver on device fields u [n_grid, nx] or
    [n_grid, nx, ny] (in place; returns u).  nu: one value per field or one
    per node."""
    torch = _torch()
    if u.dtype != torch.float64 or not u.is_contiguous():
        raise CromError("u must be a contiguous float64 tensor")
    dim = u.dim() - 1
    shape = (c_int64 * dim)(*u.shape[1:])
    nu = torch.as_tensor(nu, dtype=torch.float64, device=u.device).contiguous()
    per_node = int(nu.numel() == u.numel())
    if not per_node and nu.numel() != u.shape[0]:
        raise CromError("nu must hold one value per field or per node")
    scratch = torch.empty_like(u) if scratch is None else scratch
    _check(lib().crom_fd_heat(dim, shape, u.shape[0], _ptr(nu), per_node, dx, dt, steps, _ptr(u),
                              _ptr(scratch), _stream()), "crom_fd_heat")
    return u


# ---------------------------------------------------------------------------
# Robust sample selection (Appendix "Robust Sampling").
# ---------------------------------------------------------------------------
SAMPLING_MAX_TRY = 64


def sampling_residual(dec: Decoder, nodes, q, ref):
    """Residual vectors and metrics of sample sets from their final latents:
    nodes [P, m] FP32, q [n_set, n_mu, r] FP64, ref [n_mu, P, d] FP64 (all on
    the device).  Returns (res [n_set, P], metric [n_set]) FP64 tensors."""
    torch = _torch()
    dev = dec.params.device
    nodes = nodes.to(device=dev, dtype=torch.float32).contiguous()
    q = q.to(device=dev, dtype=torch.float64).contiguous()
    ref = ref.to(device=dev, dtype=torch.float64).contiguous()
    n_set, n_mu = int(q.shape[0]), int(q.shape[1])
    P = int(nodes.shape[0])
    if q.shape[2] != dec.r or ref.numel() != n_mu * P * dec.d:
        raise CromError("q must be [n_set, n_mu, r] and ref [n_mu, P, d]")
    res = torch.empty(n_set, P, dtype=torch.float64, device=dev)
    metric = torch.empty(n_set, dtype=torch.float64, device=dev)
    net = dec._net()
    _check(lib().crom_sampling_residual(ctypes.byref(net), _ptr(nodes), P, n_set, n_mu, _ptr(q), _ptr(ref),
                                        _ptr(res), _ptr(metric), _stream()), "crom_sampling_residual")
    return res, metric


def sampling_candidates(res, n: int, member=None):
    """The n nodes outside `member` (uint8 mask or None) with the largest
    residuals res [P] (FP64, device); -1 past the eligible nodes."""
    torch = _torch()
    res = res.to(torch.float64).contiguous()
    if member is not None:
        member = member.to(device=res.device, dtype=torch.uint8).contiguous()
    cand = torch.empty(n, dtype=torch.int32, device=res.device)
    _check(lib().crom_sampling_candidates(_ptr(res), res.numel(), _ptr(member), n, _ptr(cand), _stream()),
           "crom_sampling_candidates")
    return cand


@dataclass
class SamplingResult:
    samples: np.ndarray            # the set, in the order the nodes joined it
    metric: float                  # mean + max of its residual vector
    reached: bool                  # metric < target
    rounds: int
    candidates: Optional[np.ndarray] = None   # [rounds, n_try] per round (-1 padded)
    metrics: Optional[np.ndarray] = None      # [rounds, n_try] per round (NaN padded)


def robust_sampling(dec: Decoder, nodes, ref, q0, coef, dt: float, init, n_steps: int, target: float,
                    n_try: int = 10, max_samples: Optional[int] = None, opts: "GNOptions" = None,
                    pde: str = "heat", node_clamp=None, trace: bool = False) -> SamplingResult:
    """Greedy selection of integration samples from the nodes [P, m]
    (crom_robust_sampling).  ref [n_mu, P, d] full-order field at step
    n_steps per training parameter; q0 [n_mu, r] initial latents; coef per
    parameter (heat: nu [n_mu]; neo-Hookean: [n_mu, 6]); init: initial node
    indices."""
    torch = _torch()
    dev = dec.params.device
    kind = {"heat": PDE_HEAT, "neohookean": PDE_NEOHOOKEAN}[pde]
    nodes = nodes.to(device=dev, dtype=torch.float32).contiguous()
    P = int(nodes.shape[0])
    ref = ref.to(device=dev, dtype=torch.float64).contiguous()
    q0 = torch.as_tensor(q0, dtype=torch.float64).to(dev).reshape(-1, dec.r).contiguous()
    n_mu = int(q0.shape[0])
    per = 1 if kind == PDE_HEAT else 6
    coef = torch.as_tensor(coef, dtype=torch.float64).to(dev).reshape(n_mu, per).contiguous()
    if node_clamp is not None:
        node_clamp = node_clamp.to(device=dev, dtype=torch.uint8).contiguous()
    init = np.asarray(init, dtype=np.int32).ravel()
    max_samples = int(max_samples if max_samples is not None else P)
    o = CromSamplingOpts(int(n_try), max_samples, int(n_steps), float(target))
    net = dec._net()
    nbytes = c_size_t(0)
    _check(lib().crom_sampling_workspace(ctypes.byref(net), kind, n_mu, P, ctypes.byref(o), ctypes.byref(nbytes)),
           "crom_sampling_workspace")
    ws = torch.empty(int(nbytes.value) + 256, dtype=torch.uint8, device=dev)
    ws_ptr = (ws.data_ptr() + 255) // 256 * 256
    samples = np.zeros(max_samples, dtype=np.int32)
    samples[:init.size] = init
    rounds_max = max(1, max_samples - init.size)
    tc = np.full((rounds_max, n_try), -1, dtype=np.int32) if trace else None
    tm = np.full((rounds_max, n_try), np.nan) if trace else None
    g = (opts or GNOptions()).c_struct()
    pd = CromPDE(kind, 0, float(dt), coef.data_ptr(), None)
    out = CromSamplingResult()
    _check(lib().crom_robust_sampling(ctypes.byref(net), ctypes.byref(pd), n_mu, _ptr(nodes), P, _ptr(node_clamp),
                                      _ptr(ref), _ptr(q0), ctypes.byref(g), ctypes.byref(o),
                                      samples.ctypes.data_as(c_void_p), int(init.size), ctypes.byref(out),
                                      None if tc is None else tc.ctypes.data_as(c_void_p),
                                      None if tm is None else tm.ctypes.data_as(c_void_p),
                                      ws_ptr, int(nbytes.value), _stream()), "crom_robust_sampling")
    n = int(out.n_samples)
    return SamplingResult(samples[:n].copy(), float(out.metric), bool(out.reached), int(out.rounds),
                          None if tc is None else tc[:out.rounds].copy(),
                          None if tm is None else tm[:out.rounds].copy())


def kernel_timer(on: bool) -> None:
    """Start (dropping any earlier record) or stop recording the compute
    kernels of every crom_step on this thread (crom_kernel_timer)."""
    _check(lib().crom_kernel_timer(int(bool(on))), "crom_kernel_timer")


def kernel_timer_read() -> Tuple[float, int]:
    """(summed milliseconds, number of steps) of the record (synchronises)."""
    ms, n = c_double(0.0), c_int64(0)
    _check(lib().crom_kernel_timer_read(ctypes.byref(ms), ctypes.byref(n)), "crom_kernel_timer_read")
    return float(ms.value), int(n.value)
