"""torch.autograd interface to the adjoint: the outflow flux of species 1 as a
differentiable function of the nodal inflow/Dirichlet data and of Pe.

    J = DGNPObjective.apply(bc_conc, Pe, problem, solve_kw)
    J.backward()      # bc_conc.grad and Pe.grad from one transposed FGMRES solve

forward() sets the parameters and solves the nonlinear problem (dgnp_solve);
backward() calls dgnp_adjoint at the converged state, with the boundary data
and Pe that forward() used: when the shared problem has been given other
parameters in between (another forward, or set_params), backward() puts the
saved ones back first.  Only argument marshalling happens here; every step
runs in libdgnp.
"""
from __future__ import annotations

import numpy as np
import torch


class DGNPObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, bc_conc, Pe, problem, solve_kw=None):
        kw = dict(solve_kw or {})
        bc = np.array(bc_conc.detach().double().cpu().numpy(), dtype=np.float64, copy=True)
        pe = float(Pe)
        problem.set_params(bc, pe)
        x, st = problem.solve(**kw)
        if st.status != 0:
            raise RuntimeError(f"nonlinear solve failed (status {st.status})")
        ctx.problem = problem
        ctx.kw = kw
        ctx.bc_meta = (bc_conc.shape, bc_conc.dtype, bc_conc.device)
        ctx.params = (bc.reshape(problem.m - 1, problem.n_bnode), pe)
        ctx.pe_meta = (Pe.shape, Pe.dtype, Pe.device) if isinstance(Pe, torch.Tensor) else None
        ctx.save_for_backward(x)
        out_device = bc_conc.device if bc_conc.device.type == "cpu" else torch.device("cpu")
        return torch.tensor(problem.objective(x), dtype=torch.float64, device=out_device)

    @staticmethod
    def backward(ctx, gJ):
        (x,) = ctx.saved_tensors
        shape, dtype, device = ctx.bc_meta
        problem = ctx.problem
        bc, pe = ctx.params
        if not (problem.Pe == pe and problem.current_bc() is not None
                and np.array_equal(problem.current_bc(), bc)):
            problem.set_params(bc, pe)
        J, dbc, dpe, lam, st = problem.adjoint(x, **ctx.kw)
        g = float(gJ)
        dbc_t = torch.as_tensor(dbc * g, dtype=dtype, device=device).reshape(shape)
        dpe_t = None
        if ctx.pe_meta is not None:
            pshape, pdtype, pdevice = ctx.pe_meta
            dpe_t = torch.full(pshape, dpe * g, dtype=pdtype, device=pdevice)
        return dbc_t, dpe_t, None, None
