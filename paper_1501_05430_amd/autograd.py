"""Differentiable rollout: torch.autograd.Function over N time steps, backward by the library's adjoint step.

rho_N = Rollout(theta_bottom, theta_top, G) runs N steps from a fixed initial state with per-column wall angles
(radians) and returns the fluid-row density [ny-2, nx] after the last step. backward() walks the steps in reverse
with lbm_adjoint_step: the forward pass keeps an FP64 checkpoint of the populations every `seg` steps, and each
segment is recomputed (its states kept on the device) before its adjoint steps run. For an instance with FP32
storage the segment's states and the adjoints are kept in FP32 and go through lbm_adjoint_step_f32 (FP64
arithmetic, lambda rounded to FP32 once per step), unless fp32_adjoint=False asks for the FP64 entry point.

G enters the model twice (the force prefactor of Eq. 9, and of Q in Eq. 17, and the G inside the psi inversion of
Eq. 10); the library returns the two partials and, since one G feeds both, the gradient returned for G is their
sum (the chain rule of that tie). With geometric walls (or periodic rows) that total is zero: every term depends on
G only through G psi^2, which Eq. 10 fixes. With Martys-Chen walls it is not: the fluid-solid force of Eq. 14 has
its own G_w and scales with psi alone, so it changes with G. The two parts of the last backward are kept in
`Rollout.last_G_parts` = (dL/dG_f, dL/dG_psi).
"""
import numpy as np
import torch

from .lbm import LBM


class Rollout(torch.autograd.Function):
    last_G_parts = (0.0, 0.0)

    @staticmethod
    def forward(ctx, theta_bottom, theta_top, G, sim, f0, nsteps, seg, fp32_adjoint=None):
        assert isinstance(sim, LBM) and sim.params[0].enable_adjoint, "needs an LBM created with enable_adjoint"
        assert abs(float(G) - sim.params[0].G) == 0.0, "G must equal the instance's G"
        nsteps, seg = int(nsteps), int(seg)
        sim.apply_wetting(theta_bottom.detach().cpu().numpy(), theta_top.detach().cpu().numpy())
        sim.set_populations(f0)
        checkpoints = []
        done = 0
        while done < nsteps:
            checkpoints.append(sim.populations(device=True))
            k = min(seg, nsteps - done)
            sim.step(k)
            done += k
        rho = sim.rho(device=True)[1:-1].clone()
        sim.stream.synchronize()
        ctx.sim, ctx.nsteps, ctx.seg, ctx.checkpoints = sim, nsteps, seg, checkpoints
        ctx.f32 = (sim.params[0].precision != 0) if fp32_adjoint is None else bool(fp32_adjoint)
        ctx.theta = (theta_bottom.detach().cpu().numpy(), theta_top.detach().cpu().numpy())
        return rho.to(theta_bottom.device)

    @staticmethod
    def backward(ctx, grad_rho):
        sim, nsteps, seg = ctx.sim, ctx.nsteps, ctx.seg
        p = sim.params[0]
        dev = sim.device
        dtype = torch.float32 if ctx.f32 else torch.float64
        with torch.cuda.stream(sim.stream):
            g = grad_rho.detach().to(dev, torch.float64).contiguous()
            lam = torch.empty((9, p.ny - 2, p.nx), dtype=dtype, device=dev)
            lam_prev = torch.empty_like(lam)
            theta_bar = torch.empty((2, p.nx), dtype=torch.float64, device=dev)
            G_bar = torch.empty(2, dtype=torch.float64, device=dev)
        sim.adjoint_seed_rho(g, lam, theta_bar, G_bar)  # lambda_N = dL/drho_N on every population; sums zeroed
        sim.apply_wetting(*ctx.theta)
        starts = list(range(0, nsteps, seg))
        for si in reversed(range(len(starts))):
            k = min(seg, nsteps - starts[si])
            sim.set_populations(ctx.checkpoints[si])
            states = []
            for j in range(k):
                states.append(sim.populations(device=True).to(dtype))
                if j + 1 < k:
                    sim.step(1)
            for j in reversed(range(k)):
                sim.adjoint_step(states[j], lam, lam_prev, theta_bar, G_bar)
                lam, lam_prev = lam_prev, lam
        sim.stream.synchronize()
        gb = G_bar.cpu().numpy()
        Rollout.last_G_parts = (float(gb[0]), float(gb[1]))
        tb = theta_bar.cpu()
        ctx.checkpoints = None
        return (tb[0].to(grad_rho.device), tb[1].to(grad_rho.device),
                torch.tensor(float(gb[0] + gb[1]), dtype=torch.float64), None, None, None, None, None)


def rollout(theta_bottom, theta_top, G, sim, f0, nsteps, seg=100, fp32_adjoint=None):
    """fp32_adjoint: None follows the instance's storage precision; True / False force the FP32 / FP64 entry point."""
    return Rollout.apply(theta_bottom, theta_top, torch.as_tensor(G, dtype=torch.float64), sim, f0, nsteps, seg,
                         fp32_adjoint)
