"""Newton with direct sparse solves, adjoint, and error norms (test infrastructure).

* Initial guess (Sec. 4.3): constant concentrations equal to the mean of the
  inflow / Dirichlet data (1 where a manufactured solution supplies the data),
  and the potential from the charge equation at those constant concentrations
  (linear in phi), solved exactly here.
* Newton with backtracking line search (Sec. 4): delta = -J^{-1} R by SuperLU,
  Armijo test ||R(x + lam delta)|| <= (1 - 1e-4 lam) ||R(x)||, lam halved at most
  10 times; stop when ||R|| <= tol ||R_0|| or the step stalls.
* Adjoint: J^T lam = dJ/dx by the transposed LU; gradients
  dJ/dtheta = dJ/dtheta|_x - lam^T dR/dtheta for theta = boundary data and Pe,
  and the exchange currents and applied potentials of electrode faces.
* c_m recovery by electroneutrality (Eq. substitution).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from workload.configs import MMS_NONE

from .dg import DG
from .mesh import BoxMesh
from .quadrature import gauss_legendre, lagrange


def initial_guess(dg: DG) -> np.ndarray:
    P, msh = dg.P, dg.msh
    x = np.zeros((dg.m, msh.E, msh.nb))
    for k in range(1, dg.m):
        x[k] = 1.0 if P.mms != MMS_NONE else float(np.mean(P.bc_conc[k - 1]))
    xf = x.reshape(-1)
    Nf = msh.Nf
    r0 = dg.residual(xf)[:Nf]
    A = dg.jacobian(xf, fields=[(0, 0)])[:Nf, :Nf]
    x[0] = spla.splu(A.tocsc()).solve(-r0).reshape(msh.E, msh.nb)
    return x.reshape(-1)


def newton(dg: DG, x0=None, tol=1e-12, max_it=30, verbose=False):
    x = initial_guess(dg) if x0 is None else np.array(x0, float)
    r = dg.residual(x)
    r0 = np.linalg.norm(r)
    hist = [r0]
    for it in range(max_it):
        rn = np.linalg.norm(r)
        if rn <= tol * r0 or rn == 0.0:
            break
        J = dg.jacobian(x)
        delta = spla.splu(J.tocsc()).solve(-r)
        lam = 1.0
        for _ in range(11):
            xt = x + lam * delta
            rt = dg.residual(xt)
            if np.linalg.norm(rt) <= (1.0 - 1e-4 * lam) * rn:
                break
            lam *= 0.5
        step = lam * np.linalg.norm(delta)
        x, r = xt, rt
        hist.append(np.linalg.norm(r))
        if verbose:
            print(f"newton {it}: |R|={hist[-1]:.3e} lam={lam}")
        if step <= 1e-15 * max(1.0, np.linalg.norm(x)):
            break
    return x, np.array(hist)


def adjoint(dg: DG, x, kind=0):
    """Returns (J, dJ/d(boundary data) [m-1, n_bnode], dJ/dPe, lambda) of
    objective `kind` (0: outflow flux of species 1, 1: electrode current)."""
    J = dg.jacobian(x)
    gx, gPe = dg.objective_grad(x, kind)
    lam = spla.splu(J.tocsc()).solve(gx, trans="T")
    dg_data = -dg.dR_dg_T(x, lam)
    dPe = gPe - float(lam @ dg.dR_dPe(x))
    return dg.objective(x, kind), dg_data, dPe, lam


def adjoint_with_electrodes(dg: DG, x, kind=0):
    """adjoint() plus the gradients with respect to the electrode parameters
    (exchange current and applied potential of every box face)."""
    J, dg_data, dPe, lam = adjoint(dg, x, kind)
    j0, pa = dg.dR_dbv_T(x, lam)
    ej0, epa = dg.objective_dbv(x, kind)
    return J, dg_data, dPe, lam, ej0 - j0, epa - pa


def recover_cm(dg: DG, x):
    """Eliminated concentration c_m = -(1/z_m) sum_{k<m} z_k c_k at every node."""
    P = dg.P
    X = dg.fields(x)
    return -sum(P.z[k - 1] * X[k] for k in range(1, dg.m)) / P.z[dg.m - 1]


def l2_errors(dg: DG, x, extra=2):
    """L2(Omega) error of every field against the manufactured solution, with a
    Gauss rule of p + 2 + extra points per axis."""
    P, msh = dg.P, dg.msh
    nq = msh.nq + extra
    xq, wq = gauss_legendre(nq)
    V, _ = lagrange(msh.xn, xq)
    fine = BoxMesh(msh.dim, msh.n, msh.lo, msh.hi, msh.p, nq=nq)
    pts = fine.vol_points()
    X = dg.fields(x)
    errs = []
    for f in range(dg.m):
        uh = X[f] @ fine.phi.T
        ue = P.exact(f, pts)
        errs.append(float(np.sqrt(np.sum((uh - ue) ** 2 * fine.wvol[None, :]))))
    return errs
