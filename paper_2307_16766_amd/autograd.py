"""torch.autograd.Function over the library's recorded run and discrete adjoint.

``simulate(sigma, alpha, rho0, ux0, uy0, T0, ...)`` runs ``nsteps`` steps from the given initial
fields with the relaxation parameters sigma and alpha on every LODI-RELAX and CBC-RELAX side and
returns the final macroscopic fields stacked as a (4, ny, nx) float64 tensor (rho, ux, uy, T).
CBC and CBC-RELAX sides take the mesoscopic viscous terms, or with ``visc="fd"`` those of the
-FD variant (Sec. 4.2, "Treatment of viscous terms").  Its backward
calls ``lbm_adjoint`` with dL/d(output) as the seed: the gradient flows to sigma, alpha and the
four initial fields.  Forward and backward both run in the HIP library; torch supplies memory,
the stream and the autograd graph.
"""
import torch

from . import lbm


class ThermalLBMFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sigma, alpha, rho0, ux0, uy0, T0, spec):
        sim = lbm.LBM(spec["stencil"], spec["nx"], spec["ny"], spec["tau"], spec["bc"],
                      (rho0.detach(), ux0.detach(), uy0.detach(), T0.detach()), precision=spec.get("precision", "fp64"))
        relax = dict(spec.get("relax", {}))
        relax_sides = [s for s, b in enumerate(spec["bc"]) if b in ("lodi_relax", "cbc_relax")]
        for s in relax_sides:
            sim.set_relax(s, sigma=float(sigma), alpha=float(alpha), **relax)
        if spec.get("visc"):
            sim.set_viscous(-1, spec["visc"])
        sim.record(spec["nsteps"], spec.get("every", 50))
        out = torch.stack(sim.macroscopic())
        ctx.sim = sim
        ctx.relax_sides = relax_sides
        return out

    @staticmethod
    def backward(ctx, gout):
        sim = ctx.sim
        grad, grel = sim.adjoint(seed=gout.detach().to(torch.float64).contiguous())
        dsig = sum(grel[s, 0] for s in ctx.relax_sides)
        dalp = sum(grel[s, 1] for s in ctx.relax_sides)
        dev = grad.device
        sim.close()
        ctx.sim = None
        return (torch.tensor(float(dsig), dtype=torch.float64, device=dev),
                torch.tensor(float(dalp), dtype=torch.float64, device=dev),
                grad[0], grad[1], grad[2], grad[3], None)


def simulate(sigma, alpha, rho0, ux0, uy0, T0, *, stencil, nx, ny, tau, bc, nsteps, every=50, precision="fp64",
             relax=None, visc=None):
    """Final (rho, ux, uy, T) after nsteps steps, differentiable with respect to sigma, alpha
    (0-d tensors) and the initial fields ((ny, nx) tensors on the GPU)."""
    spec = dict(stencil=stencil, nx=nx, ny=ny, tau=tau, bc=list(bc), nsteps=nsteps, every=every,
                precision=precision, relax=relax or {}, visc=visc)
    return ThermalLBMFunction.apply(sigma, alpha, rho0, ux0, uy0, T0, spec)
