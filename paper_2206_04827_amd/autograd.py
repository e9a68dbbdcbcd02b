"""torch.autograd binding of the differentiated heat run.

``heat_run(T0, g, alpha, plan, dt, n_steps)`` returns the temperature after
n_steps BDF1 steps of (d_t - alpha nabla^2) T = g (Section 3) and records the
run for backpropagation: the backward pass calls the library's adjoint (the
transposed ADI solves, transposed tau right sides and transposed transforms)
and yields gradients for T0, g and alpha.  Everything runs in the library's
kernels; this module only marshals tensors.
"""

import torch

from . import CYL_SPACE_VALUE, Heat, HeatGrad


class HeatRun(torch.autograd.Function):
    @staticmethod
    def forward(ctx, T0, g, alpha, plan, dt, n_steps, checkpoint_every, adi_tol):
        heat = Heat(plan, [T0.detach().contiguous()], g.detach().contiguous(), float(alpha), dt,
                    bdf_order=1, adi_tol=adi_tol, space=CYL_SPACE_VALUE)
        grad = HeatGrad(heat, n_steps, checkpoint_every)
        grad.forward()
        ctx.grad = grad
        ctx.alpha_meta = (alpha.device, alpha.dtype, alpha.shape)
        return heat.read(CYL_SPACE_VALUE)

    @staticmethod
    def backward(ctx, T_bar):
        grad = ctx.grad
        T0_bar, g_bar, a_bar = grad.backward(T_bar.contiguous(), CYL_SPACE_VALUE)
        dev, dt, shape = ctx.alpha_meta
        a_bar = a_bar.to(device=dev, dtype=dt).reshape(shape)
        grad.close()
        grad.heat.close()
        ctx.grad = None
        return T0_bar, g_bar, a_bar, None, None, None, None, None


def heat_run(T0, g, alpha, plan, dt, n_steps, checkpoint_every=20, adi_tol=1e-12):
    """T_N of a BDF1 heat run from T0 (value space) with forcing g and
    diffusivity alpha (a 0-dim float64 tensor), differentiable in all three."""
    if not torch.is_tensor(alpha):
        alpha = torch.tensor(float(alpha), dtype=torch.float64)
    return HeatRun.apply(T0, g, alpha, plan, float(dt), int(n_steps), int(checkpoint_every),
                         float(adi_tol))
