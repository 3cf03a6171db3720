"""torch.autograd form of the differentiable segment.

`segment_loss(context, x, v, m, comp, gal, dt, nsteps, ...)` loads (x, v, m)
into an sbx context, integrates nsteps cycles of Eq. 6 with the fields of
Eqs. 1-8, and returns L = sum of 1/2 m v_z^2 over the selected component as
a 0-d tensor whose backward gives dL/dx, dL/dv, dL/dm from the library's
reverse mode.  GPU tensors go to the library and come back as device memory
(sbx_load_particles_device, sbx_adjoint_segment_device); CPU tensors take
the host entry points.  Only argument marshalling happens here.
"""
import numpy as np
import torch

from . import sbx


class _Segment(torch.autograd.Function):
    @staticmethod
    def forward(fctx, x, v, m, context, comp, gal, dt, nsteps, ckpt_every, sel_comp, sel_gal):
        n = m.shape[0]
        if x.is_cuda:
            dev = x.device
            xd = x.detach().to(torch.float64).contiguous()
            vd = v.detach().to(device=dev, dtype=torch.float64).contiguous()
            md = m.detach().to(device=dev, dtype=torch.float64).contiguous()
            cd = torch.as_tensor(comp, dtype=torch.int8, device=dev).contiguous()
            gd = torch.as_tensor(gal, dtype=torch.int8, device=dev).contiguous()
            gx, gv, gm = torch.empty_like(xd), torch.empty_like(vd), torch.empty_like(md)
            # the library works on its own stream: inputs and allocations first
            torch.cuda.current_stream(dev).synchronize()
            context.sbx_load_particles_device(n, xd.data_ptr(), vd.data_ptr(), md.data_ptr(),
                                              cd.data_ptr(), gd.data_ptr())
            loss = context.sbx_adjoint_segment_device(dt, nsteps, ckpt_every, sel_comp, sel_gal,
                                                      gm.data_ptr(), gx.data_ptr(), gv.data_ptr())
        else:
            context.sbx_load_particles(x.detach().double().numpy(), v.detach().double().numpy(),
                                       m.detach().double().numpy(), comp, gal)
            loss, gm_, gx_, gv_ = context.sbx_adjoint_segment(dt, nsteps, ckpt_every, sel_comp,
                                                              sel_gal)
            gx, gv, gm = torch.from_numpy(gx_), torch.from_numpy(gv_), torch.from_numpy(gm_)
        fctx.save_for_backward(gx.to(x), gv.to(v), gm.to(m))
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
