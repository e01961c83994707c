"""torch.autograd wrappers of the right-hand side and of the SDC step.

Forward passes call rhs_eval / sdc_step, backward passes rhs_vjp /
sdc_step_vjp of the library (all arithmetic in the HIP kernels).  Inputs:
U, a ghosted device state [nU][nz+8][ny+8][nx+8] (FP64), and lnA, the
natural logarithms of the pre-exponential factors [nr] (FP64, any device).
Outputs are interior arrays [nU][nz][ny][nx].  The gradient with respect to
U is zero on the ghost layers: the periodic fill overwrites them, so the
outputs do not depend on their input values.
"""
import torch

from . import narrowsdc as N


def _set_lnA(lib, lnA):
    lib.set_log_prefactors(lnA.detach().to("cpu", torch.float64).numpy())


class RhsFunction(torch.autograd.Function):
    """dU/dt = rhs(U; lnA) on the interior of one periodic box."""

    @staticmethod
    def forward(ctx, U, lnA, lib, bx, parts):
        _set_lnA(lib, lnA)
        Uw = U.detach().clone()
        out = torch.empty((U.shape[0], bx.nz, bx.ny, bx.nx), dtype=torch.float64, device=U.device)
        lib.rhs_eval(bx, Uw, out, parts)
        ctx.save_for_backward(Uw, lnA)
        ctx.lib, ctx.bx, ctx.parts = lib, bx, parts
        return out

    @staticmethod
    def backward(ctx, gout):
        Uw, lnA = ctx.saved_tensors
        lib, bx = ctx.lib, ctx.bx
        _set_lnA(lib, lnA)
        Ub = torch.zeros((Uw.shape[0], bx.nz, bx.ny, bx.nx), dtype=torch.float64, device=Uw.device)
        lAb = torch.zeros(lnA.shape[0], dtype=torch.float64, device=Uw.device)
        lib.rhs_vjp(bx, Uw, gout.contiguous(), Ub, lAb, ctx.parts)
        gU = torch.zeros_like(Uw)
        N.interior(gU).copy_(Ub)
        return gU, lAb.to(lnA.device, lnA.dtype), None, None, None


class SdcStepFunction(torch.autograd.Function):
    """Interior of U_N after nsteps single-rate SDC steps of size dt from the
    ghosted U_0."""

    @staticmethod
    def forward(ctx, U0, lnA, lib, bx, dt, nsteps, sch):
        _set_lnA(lib, lnA)
        U0c = U0.detach().clone()
        UN = U0.detach().clone()
        ws, nb = N.workspace(lib, [bx], sch, device=U0.device)
        lib.sdc_step(bx, UN, dt, nsteps, sch, ws, nb)
        ctx.save_for_backward(U0c, lnA)
        ctx.lib, ctx.bx, ctx.dt, ctx.nsteps, ctx.sch = lib, bx, dt, nsteps, sch
        return N.interior(UN).contiguous()

    @staticmethod
    def backward(ctx, gUN):
        U0c, lnA = ctx.saved_tensors
        lib, bx = ctx.lib, ctx.bx
        _set_lnA(lib, lnA)
        nb = lib.vjp_workspace_size(bx, ctx.sch, ctx.nsteps)
        ws = torch.empty(max(nb // 8, 1), dtype=torch.float64, device=U0c.device)
        gin = gUN.contiguous()
        Ub = torch.empty((U0c.shape[0], bx.nz, bx.ny, bx.nx), dtype=torch.float64, device=U0c.device)
        lAb = torch.zeros(lnA.shape[0], dtype=torch.float64, device=U0c.device)
        U0w = U0c.clone()
        lib.sdc_step_vjp(bx, U0w, ctx.dt, ctx.nsteps, ctx.sch, gin, Ub, lAb, ws, nb)
        gU = torch.zeros_like(U0c)
        N.interior(gU).copy_(Ub)
        return gU, lAb.to(lnA.device, lnA.dtype), None, None, None, None, None


def rhs(lib, bx, U, lnA, parts=N.RHS_ALL):
    return RhsFunction.apply(U, lnA, lib, bx, parts)


def sdc_step(lib, bx, U0, lnA, dt, nsteps, sch):
    return SdcStepFunction.apply(U0, lnA, lib, bx, dt, nsteps, sch)
