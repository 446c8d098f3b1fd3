"""torch.autograd integration of the adjoint gradient.

``LMLFunction.apply(h, ctx, desc, x, y, est)`` returns ln L as a 0-d float64
tensor; its backward multiplies the incoming gradient by dlnL/dh, which the
library computed in the same call (sdgp_lml_grad: one assembly, one block
CG, one adjoint pass).  h is a float64 CPU tensor in the layout of
include/sdgp.h.
"""
from __future__ import annotations

import torch


class LMLFunction(torch.autograd.Function):
    @staticmethod
    def forward(fctx, h, sctx, desc, x, y, est=None):
        val, grad, _ = sctx.lml_grad(desc, x, y, h.detach().cpu().numpy(), est)
        fctx.save_for_backward(torch.from_numpy(grad).to(h.dtype))
        return torch.tensor(val, dtype=h.dtype)

    @staticmethod
    def backward(fctx, gout):
        (g,) = fctx.saved_tensors
        return gout * g, None, None, None, None, None


def lml(h, sctx, desc, x, y, est=None):
    return LMLFunction.apply(h, sctx, desc, x, y, est)
