"""torch.autograd interface to the adjoint: the outflow flux of species 1 as a
differentiable function of the nodal inflow/Dirichlet data and of Pe.

    J = DGNPObjective.apply(bc_conc, Pe, problem, solve_kw)
    J.backward()      # bc_conc.grad and Pe.grad from one transposed FGMRES solve

forward() sets the parameters and solves the nonlinear problem (dgnp_solve);
backward() calls dgnp_adjoint at the converged state.  Only argument
marshalling happens here; every step runs in libdgnp.
"""
from __future__ import annotations

import torch


class DGNPObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, bc_conc, Pe, problem, solve_kw=None):
        kw = dict(solve_kw or {})
        problem.set_params(bc_conc.detach().double().cpu().numpy(), float(Pe))
        x, st = problem.solve(**kw)
        if st.status != 0:
            raise RuntimeError(f"nonlinear solve failed (status {st.status})")
        ctx.problem = problem
        ctx.kw = kw
        ctx.bc_meta = (bc_conc.shape, bc_conc.dtype, bc_conc.device)
        ctx.save_for_backward(x)
        return torch.tensor(problem.objective(x), dtype=torch.float64)

    @staticmethod
    def backward(ctx, gJ):
        (x,) = ctx.saved_tensors
        shape, dtype, device = ctx.bc_meta
        J, dbc, dpe, lam, st = ctx.problem.adjoint(x, **ctx.kw)
        g = float(gJ)
        dbc_t = torch.as_tensor(dbc * g, dtype=dtype, device=device).reshape(shape)
        dpe_t = torch.tensor(dpe * g, dtype=torch.float64)
        return dbc_t, dpe_t, None, None
