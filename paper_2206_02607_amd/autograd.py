"""torch.autograd.Function over the decoder: forward by the fused decode
kernel (crom_decode, one call per latent), backward by crom_decode_vjp (the
hand-written reverse-mode kernels, activations recomputed)."""
from __future__ import annotations

import torch

from .crom import CromError, Decoder, decode_vjp


class DecodeFunction(torch.autograd.Function):
    """G = decode(params, q, x): G[b, p] = g(x_p, q_b) for q [B, r], x [P, m].

    `params` must be the decoder's own parameter tensor (dec.params), with its
    packed copy current (Decoder.pack after any change)."""

    @staticmethod
    def forward(ctx, params, q, x, dec: Decoder):
        if params.data_ptr() != dec.params.data_ptr():
            raise CromError("params must be the decoder's own parameter tensor")
        B, P = q.shape[0], x.shape[0]
        out = torch.empty(B, P, dec.d, dtype=torch.float32, device=x.device)
        xc = x.to(torch.float32).contiguous()
        for b in range(B):
            dec.decode(xc, q[b].detach(), out=out[b])
        ctx.save_for_backward(q, xc)
        ctx.dec = dec
        return out

    @staticmethod
    def backward(ctx, dg):
        q, x = ctx.saved_tensors
        gp, gq = decode_vjp(ctx.dec, x, q.detach().to(torch.float32), dg.contiguous())
        return gp, gq.to(q.dtype), None, None


def decode(dec: Decoder, q, x):
    """Differentiable decode with respect to dec.params and q."""
    return DecodeFunction.apply(dec.params, q, x, dec)
