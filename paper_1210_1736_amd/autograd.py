"""torch.autograd form of the differentiable segment.

`segment_loss(context, x, v, m, comp, gal, dt, nsteps, ...)` integrates
nsteps cycles of Eq. 6 with the fields of Eqs. 1-8 from (x, v, m) and
returns L = sum of 1/2 m v_z^2 over the selected component as a 0-d tensor
whose backward gives dL/dx, dL/dv, dL/dm from the library's reverse mode.

GPU tensors: the context borrows device storage (sbx_bind_device_particles)
and writes the gradients straight into device tensors
(sbx_adjoint_segment_device).  The segment advances the particles in place,
so the storage it borrows is a structure-of-arrays copy in the context's
precision, never the caller's input tensors (autograd inputs must not be
modified); that copy is the only one, and after the call it holds the state
at the end of the segment (`context.bound_state`).  CPU tensors take the
host entry points.  Only argument marshalling happens here.
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
            pt = torch.float64 if context.prec == sbx.SBX_FP64 else torch.float32
            xs = x.detach().to(dtype=pt).t().contiguous()             # 3 x n
            vs = v.detach().to(device=dev, dtype=pt).t().contiguous()
            ms = m.detach().to(device=dev, dtype=pt).contiguous()
            cd = torch.as_tensor(comp, dtype=torch.int8, device=dev).contiguous()
            gd = torch.as_tensor(gal, dtype=torch.int8, device=dev).contiguous()
            ld = torch.zeros(n, dtype=torch.uint8, device=dev)
            gx = torch.empty((n, 3), dtype=torch.float64, device=dev)
            gv = torch.empty_like(gx)
            gm = torch.empty(n, dtype=torch.float64, device=dev)
            # the library works on its own stream: inputs and allocations first
            torch.cuda.current_stream(dev).synchronize()
            context.sbx_bind_device_particles(n, xs.data_ptr(), vs.data_ptr(), ms.data_ptr(),
                                              cd.data_ptr(), gd.data_ptr(), ld.data_ptr())
            # the storage stays borrowed by the context: keep it alive with it
            context.bound_state = {"x": xs, "v": vs, "m": ms, "comp": cd, "gal": gd, "lost": ld}
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
