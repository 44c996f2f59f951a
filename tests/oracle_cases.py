"""Small oracle problems shared by the CPU pin tests."""
import sympy as sp

from oracle.dg import DG
from oracle.problem import Problem
from workload import boundary_data, get_config
from workload.configs import (C_DIRICHLET, C_ELECTRODE, C_INFLOW, C_OUTFLOW, J0_PARABOLIC_Z, PHI_DIRICHLET,
                              VEL_CONST, VEL_POISEUILLE_X, Config)

X, Y, Z = sp.symbols("x y z")


def make(name, **kw):
    cfg = get_config(name).with_(**kw) if kw else get_config(name)
    prob = Problem(cfg) if cfg.mms else Problem(cfg, boundary_data(cfg))
    return DG(prob)


def adj2d():
    """2-D analogue of the adjoint cube: vortex flow, three ions, Dirichlet data
    and phi = 0.05 at x = 0, outflow and phi = 0 at x = 1, walls elsewhere."""
    cfg = get_config("cfg2").with_(name="adj2d", dim=2, n=(6, 6), lo=(0.0, 0.0), hi=(1.0, 1.0),
                                   Pe=100.0, c_bc=(C_DIRICHLET, C_OUTFLOW, 0, 0),
                                   phi_bc=(PHI_DIRICHLET, PHI_DIRICHLET, 0, 0),
                                   phi_val=(0.05, 0.0, 0.0, 0.0))
    return cfg


def poly_problem(dim=2, p=2, n=None):
    """Exact solution inside V_h (linear concentrations, bilinear potential),
    constant velocity, three ions, all boundaries Dirichlet."""
    n = n or ((4, 3) if dim == 2 else (3, 2, 2))
    cfg = Config("poly", dim, n, (0.0,) * dim, (1.0, 0.8, 0.6)[:dim], p, (1.0, -1.0, 2.0),
                 (1.0, 1.5, 0.7), VEL_CONST, 1.0, (1,) * (2 * dim), (1,) * (2 * dim),
                 (0.0,) * (2 * dim), vel_param=(0.3, -0.2, 0.1))
    if dim == 2:
        ex = [0.1 * X * Y + 0.05 * X, 1 + X / 2 + Y / 4, 1.2 - 0.3 * X + 0.2 * Y]
    else:
        ex = [0.1 * X * Y + 0.05 * X - 0.02 * Y * Z, 1 + X / 2 + Y / 4 - Z / 8,
              1.2 - 0.3 * X + 0.2 * Y + 0.1 * Z]
    return DG(Problem(cfg, exact_exprs=ex))


def bv2d(ion=1, **kw):
    """2-D channel with Butler-Volmer electrodes at y = 0 (anode) and y = 0.5
    (cathode), three ions, Poiseuille flow; the potential is free everywhere."""
    base = dict(c_bc=(C_INFLOW, C_OUTFLOW, C_ELECTRODE, C_ELECTRODE), phi_bc=(0, 0, 0, 0),
                phi_val=(0.0,) * 4, bv_ion=ion, bv_alpha=(1.0, 1.0), bv_j0=(0.0, 0.0, 1.0, 1.0),
                bv_phi_app=(0.0, 0.0, 0.0, 1.1676))
    base.update(kw)
    return Config("bv2d", 2, (6, 4), (0.0, 0.0), (1.0, 0.5), 2, (1.0, -1.0, 2.0), (1.0, 1.5, 0.7),
                  VEL_POISEUILLE_X, 100.0, seed=5, **base)


def bv3t(ion=1, p=2, **kw):
    """3-D channel with Butler-Volmer electrodes at y = 0 and y = 0.5, the
    exchange current parabolic across z, three ions, Poiseuille flow."""
    base = dict(c_bc=(C_INFLOW, C_OUTFLOW, C_ELECTRODE, C_ELECTRODE, 0, 0), phi_bc=(0,) * 6,
                phi_val=(0.0,) * 6, bv_ion=ion, bv_alpha=(1.0, 1.0), bv_j0=(0.0, 0.0, 1.0, 1.0, 0.0, 0.0),
                bv_phi_app=(0.0, 0.0, 0.0, 1.1676, 0.0, 0.0), bv_j0_profile=J0_PARABOLIC_Z)
    base.update(kw)
    return Config("bv3t", 3, (4, 2, 2), (0.0, 0.0, 0.0), (1.0, 0.5, 0.25), p, (1.0, -1.0, 2.0), (1.0, 1.5, 0.7),
                  VEL_POISEUILLE_X, 100.0, seed=6, **base)


def gmg_box(dim=2, n=(8, 8), p=1, Pe=1.0, seed=9):
    """Box with inflow data at x = 0, outflow at x = 1, walls elsewhere, the
    potential fixed on both x faces, constant velocity along x: the
    concentration blocks are convection-diffusion operators whose convection
    strength Pe sets."""
    wall = (0,) * (2 * dim - 2)
    return Config("gmgbox", dim, tuple(n), (0.0,) * dim, (1.0,) * dim, p, (1.0, -1.0, 2.0), (1.0, 1.5, 0.7),
                  VEL_CONST, Pe, (C_INFLOW, C_OUTFLOW) + wall, (PHI_DIRICHLET, PHI_DIRICHLET) + wall,
                  (0.05, 0.0) + (0.0,) * (2 * dim - 2), vel_param=(1.0, 0.0, 0.0), seed=seed)
