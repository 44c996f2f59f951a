"""Pins of the oracle's Butler-Volmer electrode terms (Sec. 2.1 Eqs. electrode
and bv, nondimensional form of Sec. 2.3, the electrode terms of Eqs. NPDG and
chargeDG) against what the continuous problem fixes.

* Consistency: a solution that is linear in y satisfies the electrode flux
  conditions on the face y = 0 exactly when its slopes solve the two flux
  equations there (species of the reacting ion, and the charge flux, which
  carries z_r g); the discrete residual then vanishes at its interpolant and
  Newton returns it.  With zero exponents the rate is the linear-kinetics limit
  g = J0 (1 - c_r), a linear Robin condition.
* Jacobian and parameter derivatives against central differences.
* Charge balance: with no potential-Dirichlet face, the charge equation tested
  with v = 1 says that the electrode currents z_r g cancel over the boundary.
* Adjoint gradients with respect to the exchange currents and applied
  potentials against central differences of full solves.
"""
import numpy as np
import pytest
import sympy as sp

from oracle import solve
from oracle.dg import DG
from oracle.problem import Problem
from tests.oracle_cases import bv2d
from workload import boundary_data, random_state, random_vector
from workload.configs import (C_DIRICHLET, C_ELECTRODE, C_INFLOW, C_OUTFLOW, PHI_DIRICHLET, VEL_CONST,
                              VEL_POISEUILLE_X, Config)

X, Y = sp.symbols("x y")


def _interp(dg):
    pts = dg.msh.node_points()
    return np.concatenate([dg.P.exact(f, pts).reshape(-1) for f in range(dg.m)])


@pytest.mark.parametrize("alpha", [(0.0, 0.0), (1.0, 0.5)])
@pytest.mark.parametrize("ion", [1, 2])
def test_linear_solution_satisfying_the_electrode_condition(alpha, ion):
    z1, z2, D1, D2 = 1.0, -1.0, 1.0, 1.5
    a1 = z1 * (D1 - D2)
    b1 = z1 * (z1 * D1 - z2 * D2)
    c0, phi0, j0, phi_app = 1.2, 0.1, 0.7, 0.4
    eta = phi_app - phi0
    c_r = c0 if ion == 1 else -z1 * c0 / z2        # the eliminated ion by electroneutrality
    g = j0 * (np.exp(alpha[0] * eta) - c_r * np.exp(-alpha[1] * eta))
    z_r = z1 if ion == 1 else z2
    # outward normal -y: species flux (D1 c1' + z1 D1 c1 phi') . n = g_1, charge
    # flux (a1 c1' + kappa phi') . n = z_r g, with c1 = c0 + beta y, phi = phi0 + phi1 y
    A = np.array([[-D1, -z1 * D1 * c0], [-a1, -b1 * c0]])
    rhs = np.array([g if ion == 1 else 0.0, z_r * g])
    beta, phi1 = np.linalg.solve(A, rhs)
    cfg = Config("bvlin", 2, (3, 2), (0.0, 0.0), (1.0, 0.8), 2, (z1, z2), (D1, D2), VEL_CONST, 1.0,
                 (C_DIRICHLET, C_DIRICHLET, C_ELECTRODE, C_DIRICHLET),
                 (PHI_DIRICHLET, PHI_DIRICHLET, 0, PHI_DIRICHLET), (0.0,) * 4,
                 vel_param=(0.3, 0.0, 0.0), bv_ion=ion, bv_alpha=alpha, bv_j0=(0.0, 0.0, j0, 0.0),
                 bv_phi_app=(0.0, 0.0, phi_app, 0.0))
    ex = [phi0 + float(phi1) * Y, c0 + float(beta) * Y]
    dg = DG(Problem(cfg, exact_exprs=ex))
    x = _interp(dg)
    r = dg.residual(x)
    scale = np.abs(dg.residual(np.zeros_like(x))).max()
    assert np.abs(r).max() <= 1e-12 * scale, np.abs(r).max() / scale
    xs, _ = solve.newton(dg, tol=1e-13)
    assert np.abs(xs - x).max() < 1e-10
    # a slope off by 1% leaves a residual: the electrode term is what balances it
    ex_bad = [phi0 + float(phi1) * Y, c0 + 1.01 * float(beta) * Y]
    dgb = DG(Problem(cfg, exact_exprs=ex_bad))
    assert np.abs(dgb.residual(_interp(dgb))).max() > 1e-6 * scale


@pytest.mark.parametrize("ion", [1, 3])
def test_bv_jacobian_matches_central_differences(ion):
    cfg = bv2d(ion)
    dg = DG(Problem(cfg, boundary_data(cfg)))
    x = random_state(cfg)
    v = random_vector(cfg)
    jv = dg.jac_apply(x, v)
    fd = (dg.residual(x + 1e-6 * v) - dg.residual(x - 1e-6 * v)) / 2e-6
    assert np.linalg.norm(fd - jv) <= 1e-8 * np.linalg.norm(jv)
    J = dg.jacobian(x)
    assert np.linalg.norm(J @ v - jv) <= 1e-13 * np.linalg.norm(jv)
    # the electrode terms matter: without them the Jacobian differs
    cw = cfg.with_(c_bc=(C_INFLOW, C_OUTFLOW, 0, 0))
    assert np.linalg.norm(DG(Problem(cw, boundary_data(cw))).jac_apply(x, v) - jv) > 1e-3 * np.linalg.norm(jv)


@pytest.mark.parametrize("ion", [1, 3])
def test_bv_parameter_derivatives(ion):
    cfg = bv2d(ion)
    data = boundary_data(cfg)
    dg = DG(Problem(cfg, data))
    x = random_state(cfg)
    lam = random_vector(cfg, 11)
    dj0, dpa = dg.dR_dbv_T(x, lam)
    for t in (2, 3):
        h = 1e-5
        j0p, j0m = list(cfg.bv_j0), list(cfg.bv_j0)
        j0p[t] += h
        j0m[t] -= h
        fd = (DG(Problem(cfg.with_(bv_j0=tuple(j0p)), data)).residual(x)
              - DG(Problem(cfg.with_(bv_j0=tuple(j0m)), data)).residual(x)) / (2 * h)
        assert abs(lam @ fd - dj0[t]) <= 1e-9 * max(abs(dj0[t]), 1e-30)
        pap, pam = list(cfg.bv_phi_app), list(cfg.bv_phi_app)
        pap[t] += h
        pam[t] -= h
        fd = (DG(Problem(cfg.with_(bv_phi_app=tuple(pap)), data)).residual(x)
              - DG(Problem(cfg.with_(bv_phi_app=tuple(pam)), data)).residual(x)) / (2 * h)
        assert abs(lam @ fd - dpa[t]) <= 1e-8 * max(abs(dpa[t]), 1e-30)
    assert dj0[0] == 0.0 and dpa[1] == 0.0


@pytest.mark.parametrize("ion", [1, 3])
def test_bv_charge_balance_and_adjoint(ion):
    cfg = bv2d(ion)
    data = boundary_data(cfg)
    dg = DG(Problem(cfg, data))
    x, hist = solve.newton(dg, tol=1e-13)
    assert hist[-1] <= 1e-12 * hist[0]
    cur = dg.electrode_currents(x)
    z_r = cfg.z[ion - 1]
    # the charge equation tested with v = 1: the electrode currents cancel
    assert abs(z_r * (cur[2] + cur[3])) <= 1e-9 * abs(cur[2])
    assert abs(cur[2]) > 1e-3
    Nf = dg.msh.Nf
    assert abs(dg.residual(x)[:Nf].sum()) <= 1e-12 * np.abs(dg.residual(x)[:Nf]).max() + 1e-13
    # with one reacting ion the electrode currents cancel, so every species
    # leaves as much as enters: the outflow objective does not depend on the
    # electrode parameters at all
    J, _, _, lam, dj0, dpa = solve.adjoint_with_electrodes(dg, x, 0)
    assert np.abs(dj0).max() <= 1e-12 * abs(J) and np.abs(dpa).max() <= 1e-12 * abs(J)
    # adjoint gradients of the anode's current (objective 1) with respect to
    # the exchange currents and applied potentials
    J, _, dpe, lam, dj0, dpa = solve.adjoint_with_electrodes(dg, x, 1)
    assert abs(J - cur[2]) <= 1e-14 * abs(J)

    def J_at(**kw):
        d2 = DG(Problem(cfg.with_(**kw), data))
        xx, _ = solve.newton(d2, tol=1e-13)
        return d2.objective(xx, 1)

    for t in (2, 3):
        h = 1e-6
        jp, jm = list(cfg.bv_j0), list(cfg.bv_j0)
        jp[t] += h
        jm[t] -= h
        fd = (J_at(bv_j0=tuple(jp)) - J_at(bv_j0=tuple(jm))) / (2 * h)
        assert abs(fd - dj0[t]) <= 1e-5 * abs(dj0[t])
        pp, pm = list(cfg.bv_phi_app), list(cfg.bv_phi_app)
        pp[t] += h
        pm[t] -= h
        fd = (J_at(bv_phi_app=tuple(pp)) - J_at(bv_phi_app=tuple(pm))) / (2 * h)
        assert abs(fd - dpa[t]) <= 1e-5 * abs(dpa[t])
