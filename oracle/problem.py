"""Problem data for the oracle: CNP coefficients, velocity, boundary data, sources.

Nondimensional charge-conservation Nernst-Planck model (Eqs. NP2, charge2 with
the scaling of Sec. 2.3, where mu_k F -> D_k because phi is scaled by F/RT):
  ions k = 1..m, ion m eliminated by electroneutrality (Eq. substitution),
  a_k   = z_k (D_k - D_m)                        (k < m)
  b_k   = z_k (z_k D_k - z_m D_m),  kappa(c) = sum_{k<m} b_k c_k
  q_k   = u - z_k D_k grad(phi)                   (Eq. NP2)
Manufactured sources (Sec. 5.1 style tests) are derived with SymPy from
  S_k   = -div(D_k grad c_k) + div(c_k q_k)
  S_phi = -div(sum_k a_k grad c_k + kappa grad phi).
"""
from __future__ import annotations

import numpy as np
import sympy as sp

from workload.configs import (C_DIRICHLET, C_ELECTRODE, C_INFLOW, J0_PARABOLIC_Z, MMS_NONE, MMS_PAPER3D,
                              MMS_TRIG2D, PHI_DIRICHLET, VEL_CONST, VEL_POISEUILLE_X, VEL_VORTEX, Config)

from .mesh import BoxMesh

_X = sp.symbols("x y z")


class Problem:
    def __init__(self, cfg: Config, bc_conc: np.ndarray | None = None, Pe: float | None = None,
                 mesh: BoxMesh | None = None, exact_exprs=None):
        """exact_exprs: optional SymPy expressions [phi, c_1, ..., c_{m-1}] in x, y, z
        that replace the built-in manufactured solution (all data then come from it)."""
        self.cfg = cfg
        self.dim = cfg.dim
        self.m = cfg.m
        self.z = np.array(cfg.z, float)
        self.D = np.array(cfg.D, float)
        self.Pe = float(cfg.Pe if Pe is None else Pe)
        self.mesh = mesh if mesh is not None else BoxMesh(cfg.dim, cfg.n, cfg.lo, cfg.hi, cfg.p)
        m = self.m
        zm, Dm = self.z[m - 1], self.D[m - 1]
        self.a = np.array([self.z[k] * (self.D[k] - Dm) for k in range(m - 1)])
        self.b = np.array([self.z[k] * (self.z[k] * self.D[k] - zm * Dm) for k in range(m - 1)])
        self.delta = cfg.c_ip * cfg.p ** 2 / self.mesh.diameter      # Eq. deltap, h = diameter
        self.c_bc = list(cfg.c_bc[: 2 * self.dim])
        self.phi_bc = list(cfg.phi_bc[: 2 * self.dim])
        self.phi_val = list(cfg.phi_val[: 2 * self.dim])
        self.mms = cfg.mms if exact_exprs is None else -1
        # Butler-Volmer electrodes (Sec. 2.1 Eq. bv, nondimensional form of Sec. 2.3)
        self.bv_ion = int(cfg.bv_ion)
        self.bv_alpha = tuple(float(a) for a in cfg.bv_alpha)
        self.bv_j0 = [float(v) for v in cfg.bv_j0[: 2 * self.dim]]
        self.bv_phi_app = [float(v) for v in cfg.bv_phi_app[: 2 * self.dim]]
        self.bv_profile = int(cfg.bv_j0_profile)
        if any(t == C_ELECTRODE for t in self.c_bc):
            if not 1 <= self.bv_ion <= m:
                raise ValueError("reacting ion must be one of the m ions")
            if any(self.c_bc[t] == C_ELECTRODE and self.phi_bc[t] == PHI_DIRICHLET for t in range(2 * self.dim)):
                raise ValueError("the potential is free on an electrode face")
        self._build_velocity()
        if self.mms != MMS_NONE:
            self._build_mms(exact_exprs)
        self.bc_conc = None
        if self.mms == MMS_NONE:
            if bc_conc is None:
                raise ValueError("boundary data required")
            self.bc_conc = np.asarray(bc_conc, float).reshape(m - 1, -1)
        self._bnode_offsets()

    # ---- velocity -----------------------------------------------------
    def _build_velocity(self):
        cfg = self.cfg
        x, y, z = _X
        if cfg.vel_kind == VEL_VORTEX:
            uh = [sp.sin(sp.pi * x) * sp.cos(sp.pi * y), -sp.cos(sp.pi * x) * sp.sin(sp.pi * y), 0]
        elif cfg.vel_kind == VEL_POISEUILLE_X:
            H = cfg.hi[1] - cfg.lo[1]
            yy = y - cfg.lo[1]
            uh = [6 * yy * (H - yy) / H ** 2, 0, 0]
        elif cfg.vel_kind == VEL_CONST:
            uh = [sp.Float(v) for v in cfg.vel_param]
        else:
            raise ValueError("velocity kind")
        self.uhat_sym = [sp.sympify(c) for c in uh[: self.dim]]
        self._uhat_f = [sp.lambdify(_X[: self.dim], c, "numpy") for c in self.uhat_sym]

    def uhat(self, pts):
        """Unit-Pe velocity at points (..., d) -> (..., d)."""
        cols = [pts[..., i] for i in range(self.dim)]
        return np.stack([np.broadcast_to(np.asarray(f(*cols), float), pts.shape[:-1])
                         for f in self._uhat_f], axis=-1)

    def u(self, pts):
        return self.Pe * self.uhat(pts)

    # ---- manufactured solutions --------------------------------------
    def _build_mms(self, exprs=None):
        x, y, z = _X[0], _X[1], _X[2]
        if exprs is not None:
            ph, cs = exprs[0], list(exprs[1:])
        elif self.mms == MMS_TRIG2D:
            cs = [1 + sp.Rational(1, 2) * sp.sin(sp.pi * x) * sp.sin(sp.pi * y)]
            ph = sp.Rational(1, 10) * sp.cos(sp.pi * x) * sp.cos(sp.pi * y)
        elif self.mms == MMS_PAPER3D:
            cs = [sp.cos(x) + sp.sin(y) + 3]
            ph = sp.sin(x) + sp.cos(y) + 3
        else:
            raise ValueError("mms kind")
        if len(cs) != self.m - 1:
            raise ValueError("one expression per unknown concentration required")
        X = _X[: self.dim]
        grad = lambda f: [sp.diff(f, v) for v in X]
        div = lambda F: sum(sp.diff(F[i], X[i]) for i in range(self.dim))
        u = [self.Pe * c for c in self.uhat_sym]
        S = []
        for k, ck in enumerate(cs):
            Dk, zk = sp.Float(self.D[k]), sp.Float(self.z[k])
            qk = [u[i] - zk * Dk * grad(ph)[i] for i in range(self.dim)]
            S.append(-div([Dk * g for g in grad(ck)]) + div([ck * qk[i] for i in range(self.dim)]))
        kap = sum(sp.Float(self.b[k]) * ck for k, ck in enumerate(cs))
        cur = [sum(sp.Float(self.a[k]) * grad(ck)[i] for k, ck in enumerate(cs)) + kap * grad(ph)[i]
               for i in range(self.dim)]
        S_p = -div(cur)
        lam = lambda f: sp.lambdify(X, f, "numpy")
        self._ex = [lam(ph)] + [lam(ck) for ck in cs]
        self._src = [lam(S_p)] + [lam(s) for s in S]

    def exact(self, f, pts):
        cols = [pts[..., i] for i in range(self.dim)]
        return np.broadcast_to(np.asarray(self._ex[f](*cols), float), pts.shape[:-1]).copy()

    def source(self, f, pts):
        """Volume source of field f (0: charge equation, k: species k) at points."""
        if self.mms == MMS_NONE:
            return np.zeros(pts.shape[:-1])
        cols = [pts[..., i] for i in range(self.dim)]
        return np.broadcast_to(np.asarray(self._src[f](*cols), float), pts.shape[:-1]).copy()

    # ---- boundary data -------------------------------------------------
    def _bnode_offsets(self):
        """Offset of each data-carrying box face in the canonical boundary-node list."""
        msh = self.mesh
        nfn = msh.nn ** (self.dim - 1)
        self.bnode_off = {}
        off = 0
        for t in range(2 * self.dim):
            if self.c_bc[t] in (C_DIRICHLET, C_INFLOW):
                self.bnode_off[t] = off
                off += len(msh.bfaces[t]) * nfn
        self.n_bnode = off

    def c_data(self, k, t):
        """Concentration data g_k (k = 1..m-1) at the Gauss points of the boundary
        faces with tag t: interpolated nodal data, or the exact solution (MMS)."""
        msh = self.mesh
        a, s = divmod(t, 2)
        side = -1 if s == 0 else 1
        elems = msh.bfaces[t]
        if self.mms != MMS_NONE:
            return self.exact(k, msh.face_points(elems, a, side))
        nfn = msh.nn ** (self.dim - 1)
        off = self.bnode_off[t]
        g = self.bc_conc[k - 1, off: off + len(elems) * nfn].reshape(len(elems), nfn)
        return g @ msh.fpsi[a].T

    def phi_data(self, t):
        msh = self.mesh
        a, s = divmod(t, 2)
        side = -1 if s == 0 else 1
        elems = msh.bfaces[t]
        if self.mms != MMS_NONE:
            return self.exact(0, msh.face_points(elems, a, side))
        nqf = msh.fw[a].shape[0]
        return np.full((len(elems), nqf), float(self.phi_val[t]))

    def is_phi_dirichlet(self, t):
        return self.phi_bc[t] == PHI_DIRICHLET

    def j0_profile(self, pts):
        """Shape of the exchange current across the box in z at points (..., d):
        1, or the parabola of Sec. 5.2 with mean 1 over the z extent."""
        if self.bv_profile != J0_PARABOLIC_Z or self.dim < 3:
            return np.ones(pts.shape[:-1])
        zc = 0.5 * (self.cfg.lo[2] + self.cfg.hi[2])
        half = 0.5 * (self.cfg.hi[2] - self.cfg.lo[2])
        return 0.6 * (2.0 - ((pts[..., 2] - zc) / half) ** 2)

    def bv_data(self, t):
        """(exchange current, applied potential) at the Gauss points of the
        boundary faces with tag t (an electrode face)."""
        msh = self.mesh
        a, s = divmod(t, 2)
        pts = msh.face_points(msh.bfaces[t], a, -1 if s == 0 else 1)
        return self.bv_j0[t] * self.j0_profile(pts), np.full(pts.shape[:-1], self.bv_phi_app[t])
