"""Differentiable rollout of quasi-static projection steps (torch.autograd).

`ProjectionRollout.apply(chi0, v0, sigma0, solver, params, dt, U, nsteps, rtol,
max_cycles)`
runs `nsteps` projection steps on the GPU (qs_projection_step) and returns
the final (sigma, chi, v).  The forward pass keeps one checkpoint (v^n,
sigma^n, chi^n) per step; the backward pass walks the steps in reverse with
the library's hand-written adjoint kernels:

  s^{n+1} = s* + dt C : sym(G_h v^{n+1})   ->  qs_stress_update_vjp
  K v^{n+1} = D_h s* / dt                  ->  qs_mg_solve with K^T = K, zero walls
                                               then qs_rhs_vjp
  (s*, chi^{n+1}) = STZ(G_h v^n, s^n, chi^n) ->  qs_stz_step_vjp

Gradients are returned for chi0, sigma0 and the interior of v0 (its wall
planes are boundary data).  The plastic rate has a kink at sbar = s_Y; the
derivative of the elastic branch is used there.  rtol <= 0 runs every solve
(forward and adjoint) for exactly max_cycles V-cycles, which makes the
discrete map a smooth function of its inputs (useful for finite-difference
checks, where a residual-based stop adds noise of order cond(K) * rtol).
"""
from __future__ import annotations

import torch


class ProjectionRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, chi0, v0, sigma0, solver, params, dt, U, nsteps, rtol, max_cycles=200):
        v, s, c = v0.detach().clone(), sigma0.detach().clone(), chi0.detach().clone()
        ckpt = []
        for _ in range(nsteps):
            ckpt.append((v.clone(), s.clone(), c.clone()))
            solver.projection_step(params, dt, U, v, s, c, rtol=rtol, max_cycles=max_cycles)
        ctx.ckpt = ckpt
        ctx.solver, ctx.params, ctx.dt, ctx.rtol = solver, params, dt, rtol
        ctx.max_cycles = max_cycles
        return s, c, v

    @staticmethod
    def backward(ctx, g_s, g_c, g_v):
        solver, params, dt, rtol = ctx.solver, ctx.params, ctx.dt, ctx.rtol
        shape_v = solver.node_shape()
        g_s = torch.zeros_like(ctx.ckpt[0][1]) if g_s is None else g_s.contiguous().clone()
        g_c = torch.zeros_like(ctx.ckpt[0][2]) if g_c is None else g_c.contiguous().clone()
        g_v = (torch.zeros(shape_v, dtype=torch.float64, device=solver.device) if g_v is None
               else g_v.contiguous().clone())
        for n in reversed(range(len(ctx.ckpt))):
            vn, sn, cn = ctx.ckpt[n]
            g_sstar = g_s.clone()
            solver.stress_update_vjp(g_s, dt, g_v)
            g_v[:, 0].zero_()
            g_v[:, -1].zero_()
            lam_v = torch.zeros_like(g_v)
            solver.solve(g_v, lam_v, rtol=rtol, max_cycles=ctx.max_cycles)
            solver.rhs_vjp(lam_v, dt, g_sstar)
            g_v = torch.zeros_like(g_v)
            g_s, g_c = solver.stz_step_vjp(params, dt, vn, sn, cn, g_sstar, g_c, g_v)
        ctx.ckpt = None
        return g_c, g_v, g_s, None, None, None, None, None, None, None


def mid_shear_loss(sigma: torch.Tensor) -> torch.Tensor:
    """Mean of sigma_xz^2 over the two cell layers next to the plane z = 1/2."""
    nz = sigma.shape[1]
    s = sigma[4, nz // 2 - 1: nz // 2 + 1]
    return (s * s).mean()


def rollout_loss(chi0, v0, sigma0, solver, params, dt, U, nsteps, rtol=1e-12, max_cycles=200):
    s, c, v = ProjectionRollout.apply(chi0, v0, sigma0, solver, params, dt, U, nsteps, rtol,
                                      max_cycles)
    return mid_shear_loss(s)
