"""Small oracle problems shared by the CPU pin tests."""
import sympy as sp

from oracle.dg import DG
from oracle.problem import Problem
from workload import boundary_data, get_config
from workload.configs import C_DIRICHLET, C_OUTFLOW, PHI_DIRICHLET, VEL_CONST, Config

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
