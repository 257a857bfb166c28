"""torch.autograd.Function around pb_solve_dev / pb_forces_dev.

``pb_energy(verts, tris, pos, q, ctx, params)`` returns E_sol (kcal/mol) as a
0-d float64 device tensor.  The surface is held fixed; gradients flow to the
charge positions and charges.  When either needs a gradient the forward call
runs the forward and adjoint solves together (pb_forces_dev) and keeps
dE/dpos, dE/dq for the backward pass, which only scales them.  A solve that
stops before its tolerance (PB_NOT_CONVERGED) raises PbError instead of
returning an unconverged energy.
"""
from __future__ import annotations

import torch

from .pbsolve import Context, Params, PbError, PB_OK


class PBEnergy(torch.autograd.Function):
    @staticmethod
    def forward(fctx, verts, tris, pos, q, ctx: Context, params: Params):
        pos_c = pos.detach().contiguous()
        q_c = q.detach().contiguous()
        want = fctx.needs_input_grad[2] or fctx.needs_input_grad[3]
        if want:
            gpos = torch.empty_like(pos_c)
            gq = torch.empty_like(q_c)
            info = ctx.pb_forces_dev(verts, tris, pos_c, q_c, params, gpos, gq)
            fctx.save_for_backward(gpos, gq)
        else:
            info = ctx.pb_solve_dev(verts, tris, pos_c, q_c, params)
        if info.status != PB_OK:
            # an energy or gradient of an unconverged solve is not E_sol
            raise PbError(info.status,
                          f"GMRES stopped before tol {params.tol:g} (relative residual "
                          f"{info.rel_residual:.3e}, forward {info.iters} and adjoint "
                          f"{info.adjoint_iters} Arnoldi steps); raise max_iter or max_refine")
        fctx.info = info
        return torch.tensor(info.e_solv, dtype=torch.float64, device=pos.device)

    @staticmethod
    def backward(fctx, g_e):
        gpos, gq = fctx.saved_tensors
        return None, None, g_e * gpos, g_e * gq, None, None


def pb_energy(verts, tris, pos, q, ctx: Context, params: Params):
    return PBEnergy.apply(verts, tris, pos, q, ctx, params)
