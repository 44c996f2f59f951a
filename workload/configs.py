"""Problem configurations (plain data).

Box faces are tagged 0..5 = x-, x+, y-, y+, z-, z+ (tag = 2*axis + side).
Boundary kinds for the concentrations: WALL, DIRICHLET, INFLOW, OUTFLOW,
ELECTRODE (Butler-Volmer reaction of one ion, Sec. 2.1);
for the potential: NEUMANN0, DIRICHLET.  Velocity kinds: VORTEX
(u = Pe (sin pi x cos pi y, -cos pi x sin pi y, 0)), POISEUILLE_X
(u_x = 6 Pe y'(H - y')/H^2 with y' = y - y_lo and H the box height in y) and
CONST (u = Pe * param).  MMS kinds select a built-in manufactured solution:
TRIG2D (c1 = 1 + sin(pi x) sin(pi y)/2, phi = cos(pi x) cos(pi y)/10) and
PAPER3D (the paper's convergence test: c1 = cos x + sin y + 3,
phi = sin x + cos y + 3).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Tuple

C_WALL, C_DIRICHLET, C_INFLOW, C_OUTFLOW, C_ELECTRODE = 0, 1, 2, 3, 4
J0_CONST, J0_PARABOLIC_Z = 0, 1
PHI_NEUMANN0, PHI_DIRICHLET = 0, 1
VEL_VORTEX, VEL_POISEUILLE_X, VEL_CONST = 0, 1, 2
MMS_NONE, MMS_TRIG2D, MMS_PAPER3D = 0, 1, 2


@dataclass(frozen=True)
class Config:
    name: str
    dim: int
    n: Tuple[int, ...]
    lo: Tuple[float, ...]
    hi: Tuple[float, ...]
    p: int
    z: Tuple[float, ...]
    D: Tuple[float, ...]
    vel_kind: int
    Pe: float
    c_bc: Tuple[int, ...]
    phi_bc: Tuple[int, ...]
    phi_val: Tuple[float, ...]
    mms: int = MMS_NONE
    seed: int = 0
    c_ip: float = 10.0
    vel_param: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    newton_tol: float = 1e-8
    note: str = ""
    # Butler-Volmer electrodes (faces tagged C_ELECTRODE): reacting ion (1..m,
    # the oxidant; m is the eliminated ion), anodic / cathodic exponents
    # (alpha_a n, alpha_c n), exchange current and applied potential per box
    # face (nondimensional), and the exchange-current profile across z
    bv_ion: int = 1
    bv_alpha: Tuple[float, float] = (1.0, 1.0)
    bv_j0: Tuple[float, ...] = (0.0,) * 6
    bv_phi_app: Tuple[float, ...] = (0.0,) * 6
    bv_j0_profile: int = J0_CONST

    @property
    def m(self) -> int:
        return len(self.z)

    def with_(self, **kw) -> "Config":
        return replace(self, **kw)


_ION3_Z = (1.0, -1.0, 2.0)
_ION3_D = (1.0, 1.5, 0.7)

CONFIGS = {
    # 2-D manufactured solution, binary electrolyte, all boundaries Dirichlet.
    "cfg1": Config("cfg1", 2, (8, 8), (0.0, 0.0), (1.0, 1.0), 2, (1.0, -1.0), (1.0, 1.0),
                   VEL_VORTEX, 1.0, (1, 1, 1, 1), (1, 1, 1, 1), (0.0,) * 4,
                   mms=MMS_TRIG2D, newton_tol=1e-10,
                   note="2D MMS 8x8 p=2"),
    # 3-D cube, vortex flow, three ions.  x=0: Dirichlet c (seeded) and phi=0.05;
    # x=1: outflow and phi=0; y/z faces: walls with zero-Neumann potential.
    "cfg2": Config("cfg2", 3, (16, 16, 16), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), 2, _ION3_Z, _ION3_D,
                   VEL_VORTEX, 1e3, (C_DIRICHLET, C_OUTFLOW, 0, 0, 0, 0),
                   (PHI_DIRICHLET, PHI_DIRICHLET, 0, 0, 0, 0), (0.05, 0.0, 0.0, 0.0, 0.0, 0.0),
                   seed=0, note="3D cube 16^3 p=2 vortex Pe=1e3"),
    # Flow-plate channel: inflow at x=0, outflow at x=8, electrodes (fixed phi)
    # at y=0 and y=2, walls at z faces.
    "cfg3": Config("cfg3", 3, (64, 16, 8), (0.0, 0.0, 0.0), (8.0, 2.0, 1.0), 3, _ION3_Z, _ION3_D,
                   VEL_POISEUILLE_X, 1e4, (C_INFLOW, C_OUTFLOW, 0, 0, 0, 0),
                   (0, 0, PHI_DIRICHLET, PHI_DIRICHLET, 0, 0), (0.0, 0.0, 0.0, 0.1, 0.0, 0.0),
                   seed=1, note="channel 64x16x8 p=3 Poiseuille Pe=1e4"),
    "cfg5": Config("cfg5", 3, (128, 32, 16), (0.0, 0.0, 0.0), (8.0, 2.0, 1.0), 3, _ION3_Z, _ION3_D,
                   VEL_POISEUILLE_X, 1e4, (C_INFLOW, C_OUTFLOW, 0, 0, 0, 0),
                   (0, 0, PHI_DIRICHLET, PHI_DIRICHLET, 0, 0), (0.0, 0.0, 0.0, 0.1, 0.0, 0.0),
                   seed=2, note="channel 128x32x16 p=3 Poiseuille Pe=1e4"),
    # The paper's manufactured-solution convergence problem on the unit cube.
    "e1": Config("e1", 3, (4, 4, 4), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), 1, (2.0, -2.0), (5e-6, 1e-5),
                 VEL_POISEUILLE_X, 1.0, (1,) * 6, (1,) * 6, (0.0,) * 6, mms=MMS_PAPER3D,
                 newton_tol=1e-10, note="paper convergence test"),
}
# cfg4 is the adjoint study on the cfg2 cube (same data seed).
CONFIGS["cfg4"] = CONFIGS["cfg2"].with_(name="cfg4", note="adjoint on cfg2 cube")
# Small variants used where the oracle's direct solver must finish quickly.
CONFIGS["cfg2s"] = CONFIGS["cfg2"].with_(name="cfg2s", n=(8, 8, 8), note="cfg2 physics on 8^3")
CONFIGS["cfg2t"] = CONFIGS["cfg2"].with_(name="cfg2t", n=(4, 4, 4), note="cfg2 physics on 4^3")
# The channel at p = 1 with the same 12.6M DOFs as cfg5: one GPU's share (an
# eighth) of the paper's 100.7M-DOF structured p = 1 strong-scaling channel,
# where the concentration-block preconditioners ASM and GMG are compared.
CONFIGS["ch256p1"] = CONFIGS["cfg5"].with_(name="ch256p1", n=(256, 64, 32), p=1,
                                          note="channel 256x64x32 p=1 Poiseuille Pe=1e4")
CONFIGS["ch64p1"] = CONFIGS["cfg5"].with_(name="ch64p1", n=(64, 16, 8), p=1,
                                         note="channel 64x16x8 p=1 Poiseuille Pe=1e4")
CONFIGS["cfg3s"] = CONFIGS["cfg3"].with_(name="cfg3s", n=(8, 4, 2), hi=(1.0, 0.5, 0.25),
                                         note="channel physics on 8x4x2")

# Channel with Butler-Volmer electrodes (the paper's flow-plate reactor, Sec. 5.2):
# y = 0 anode (applied potential 0) and y = y_max cathode (applied potential
# 0.03 V, i.e. 0.03 F/RT = 1.1676 nondimensional), alpha_1 = alpha_2 = 0.5 and
# n = 2 (exponents alpha n = 1), the exchange current with the paper's parabolic
# profile across z; the reacting ion is the cation of the first species (a
# primary unknown: the eliminated ion's concentration (c_2 - c_1)/2 is near
# zero for inflow data drawn from U[0.5, 1.5], too little for the cathode to
# balance the anode); the potential is free (natural) on the electrodes, where
# the Butler-Volmer current fixes it.
_BV = dict(c_bc=(C_INFLOW, C_OUTFLOW, C_ELECTRODE, C_ELECTRODE, 0, 0), phi_bc=(0,) * 6,
           phi_val=(0.0,) * 6, bv_ion=1, bv_alpha=(1.0, 1.0), bv_j0=(0.0, 0.0, 1.0, 1.0, 0.0, 0.0),
           bv_phi_app=(0.0, 0.0, 0.0, 1.1676, 0.0, 0.0), bv_j0_profile=J0_PARABOLIC_Z)
CONFIGS["bv3s"] = CONFIGS["cfg3s"].with_(name="bv3s", note="BV channel 8x4x2 p=3", **_BV)
CONFIGS["bv3"] = CONFIGS["cfg3"].with_(name="bv3", note="BV channel 64x16x8 p=3", **_BV)

ADJOINT_SEED = 4
N_ADJOINT_PARAMS = 64


def get_config(name: str) -> Config:
    return CONFIGS[name]


def n_boundary_nodes(cfg: Config) -> int:
    """Number of nodal boundary-data entries per species: one per (element face on
    a DIRICHLET/INFLOW box face, face node); (p+1)^(d-1) nodes per element face."""
    tot = 0
    for t in range(2 * cfg.dim):
        if cfg.c_bc[t] in (C_DIRICHLET, C_INFLOW):
            a = t // 2
            nf = 1
            for b in range(cfg.dim):
                if b != a:
                    nf *= cfg.n[b]
            tot += nf * (cfg.p + 1) ** (cfg.dim - 1)
    return tot
