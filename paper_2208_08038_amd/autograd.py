"""torch.autograd bridge of the gradient run.

`ProbeSeries.apply(omega_c, nu, env, builder, steps, checkpoint_every)`
returns the probe series (nprobe x steps, float64, CPU) of a run of the
system that `builder(omega_c, nu, env)` creates (a `pic.Simulation` with
its probes set).  Its backward hands the series' cotangent to the
library's adjoint (pic_grad_backward: checkpointed reverse sweep on the
GPU) and returns d/d(omega_c), d/d(nu) of species 0 and d/d(env).  Any
loss written in torch on the series (e.g. objectives.transmitted_loss)
is then differentiable end to end; this module only marshals arrays.
"""
import numpy as np
import torch


class ProbeSeries(torch.autograd.Function):
    @staticmethod
    def forward(ctx, omega_c, nu, env, builder, steps, checkpoint_every):
        sim = builder(float(omega_c), float(nu), tuple(float(v) for v in env.detach().cpu()))
        sim.grad_forward(int(steps), int(checkpoint_every))
        series = sim.probes()[:, -int(steps):]
        ctx.sim = sim
        ctx.dtype = omega_c.dtype
        return torch.from_numpy(np.ascontiguousarray(series))

    @staticmethod
    def backward(ctx, grad_series):
        sim = ctx.sim
        g = sim.grad_backward(grad_series.detach().cpu().double().numpy())
        sim.close()
        ctx.sim = None
        d_wc = torch.tensor(g["d_omega_c"][0], dtype=ctx.dtype)
        d_nu = torch.tensor(g["d_nu"][0], dtype=ctx.dtype)
        d_env = torch.from_numpy(g["d_env"]).to(ctx.dtype)
        return d_wc, d_nu, d_env, None, None, None
