"""torch.autograd.Function over the library's forward and backward applies.

LiouvilleApply.apply(a, c_occ, op) returns la = L(c_occ) a for trial
coefficients a [nb][nocc][npw][2] (context dtype) and occupied coefficients
c_occ [nocc][npw][2] (float64); gradients flow to both.  The operator object
`op` (a wtd.Liouville context) is re-pointed at c_occ with wtd_set_occ before
every call; all arithmetic happens in the HIP library.
"""
from __future__ import annotations

import torch


class LiouvilleApply(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a, c_occ, op):
        op.set_occ(c_occ.detach())
        la = op.apply(a.detach().contiguous())
        ctx.op = op
        ctx.save_for_backward(a, c_occ)
        return la

    @staticmethod
    def backward(ctx, g_la):
        a, c_occ = ctx.saved_tensors
        op = ctx.op
        want_a, want_occ = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (want_a or want_occ):
            return None, None, None
        op.set_occ(c_occ.detach())
        g = g_la.detach().to(dtype=op.dtype).contiguous()
        ga, go = op.apply_bwd(a.detach().contiguous(), g, want_a=want_a, want_occ=want_occ)
        if go is not None:
            go = go.to(dtype=c_occ.dtype)
        return ga, go, None


def liouville_apply(a, c_occ, op):
    return LiouvilleApply.apply(a, c_occ, op)
