"""torch.autograd.Function around the march: receiver values as a function of
the spring stiffnesses and positions, with the backward pass computed by the
library's gradient pass (wfp_adjoint).  Argument marshalling only."""
import torch

from . import wfp


class WFPReceivers(torch.autograd.Function):
    """u = WFPReceivers.apply(beta, x, problem, dt, n_steps, checkpoint_every)

    beta, x     float64 tensors [M] (the values used to build the plan; any
                device, copied to the host for plan creation)
    problem     dict with packets, x_recv, boundary (periodic box only for the
                backward pass)
    checkpoint_every  > 0: march-state checkpoints every that many levels
                (the backward pass replays each segment); -C < 0: every level
                recorded in blocks of C (16 M bytes per level, no replay)
    returns     float64 CUDA tensor [n_steps][R]: u(x_r, t_L), L = 0..n_steps-1
    """

    @staticmethod
    def forward(ctx, beta, x, problem, dt, n_steps, checkpoint_every=250):
        prob = dict(problem)
        prob["beta"] = beta.detach().double().cpu().numpy()
        prob["x"] = x.detach().double().cpu().numpy()
        plan = wfp.Plan(prob, dt, checkpoint_every=int(checkpoint_every))
        R = plan.info["R"]
        u = torch.empty((n_steps, R), dtype=torch.float64, device="cuda")
        plan.run(n_steps, None, 1, u)
        ctx.plan = plan
        ctx.want_x = x.requires_grad
        ctx.devices = (beta.device, x.device)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        plan = ctx.plan
        gb, gx = plan.gradient(grad_u.contiguous().double(), positions=ctx.want_x)
        plan.close()
        ctx.plan = None
        gb = gb.to(ctx.devices[0])
        gx = None if gx is None else gx.to(ctx.devices[1])
        return gb, gx, None, None, None, None
