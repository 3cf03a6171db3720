"""torch.autograd form of the differentiable segment.

`segment_loss(context, x, v, m, dt, nsteps, ...)` loads (x, v, m) into an
sbx context, integrates nsteps cycles of Eq. 6 with the fields of Eqs. 1-8,
and returns L = sum of 1/2 m v_z^2 over the selected component as a 0-d
tensor whose backward gives dL/dx, dL/dv, dL/dm from the library's reverse
mode (sbx_adjoint_segment).  Only argument marshalling happens here.
"""
import numpy as np
import torch

from . import sbx


class _Segment(torch.autograd.Function):
    @staticmethod
    def forward(fctx, x, v, m, context, comp, gal, dt, nsteps, ckpt_every, sel_comp, sel_gal):
        context.sbx_load_particles(x.detach().cpu().double().numpy(), v.detach().cpu().double().numpy(),
                                   m.detach().cpu().double().numpy(), comp, gal)
        loss, gm, gx, gv = context.sbx_adjoint_segment(dt, nsteps, ckpt_every, sel_comp, sel_gal)
        fctx.save_for_backward(torch.from_numpy(gx).to(x), torch.from_numpy(gv).to(v),
                               torch.from_numpy(gm).to(m))
        return torch.tensor(loss, dtype=torch.float64, device=x.device)

    @staticmethod
    def backward(fctx, g):
        gx, gv, gm = fctx.saved_tensors
        g = g.to(gx)
        return g * gx, g * gv, g * gm, None, None, None, None, None, None, None, None


def segment_loss(context, x, v, m, comp, gal, dt, nsteps, ckpt_every=2, sel_comp=0, sel_gal=0):
    """Loss of a segment as a differentiable function of (x, v, m)."""
    comp = np.ascontiguousarray(comp, dtype=np.int8)
    gal = np.ascontiguousarray(gal, dtype=np.int8)
    return _Segment.apply(x, v, m, context, comp, gal, float(dt), int(nsteps), int(ckpt_every),
                          int(sel_comp), int(sel_gal))
