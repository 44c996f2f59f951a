"""Residual and exact Jacobian of the DG scheme (test infrastructure).

The scheme is Eqs. NPDG and chargeDG (Sec. 3.3) in nondimensional form, with
these readings of passages the paper leaves open:
  * interior faces use n = n^- (from the lower element to the upper one),
    [w] = w^- - w^+, {w} = (w^- + w^+)/2;
  * upwind flux {c q}.n + |{q}.n| [c]/2 with {q} = u - z D {grad phi} (Sec. 3.2);
  * penalty delta = C_IP p^2 / h with h the cell diameter (Eq. deltap);
  * kappa depends on the concentrations, kappa = sum_k b_k c_k (Eq. charge2);
  * weak Dirichlet data: SIPG consistency/symmetry/penalty with exterior value g
    and an upwind boundary flux (q.n)^+ c + (q.n)^- g for the concentrations;
    consistency term with the full current sum a grad c + kappa grad phi, plus
    symmetry/penalty on phi-Dirichlet faces; a_k-symmetry on c-Dirichlet faces;
  * INFLOW faces carry (u.n) c_in v; OUTFLOW faces (q.n) c v (the scheme's form,
    Eq. NPDG); walls carry nothing; the charge equation gets no inflow/outflow
    term (the inlet terms cancel by electroneutrality);
  * ELECTRODE faces carry the reaction rate of Eq. electrode: -g v in the
    equation of the reacting ion r and -z_r g v in the charge equation (the
    current sum_k z_k g_k of Eq. chargeDG), with the Butler-Volmer rate of
    Eq. bv in the nondimensional form of Sec. 2.3, gamma = 1 and a reductant of
    constant concentration (Sec. 5.2):
      g = J0 [exp(alpha_a n (phi_app - phi)) - c_r exp(-alpha_c n (phi_app - phi))];
    c_r follows Eq. substitution when r is the eliminated ion.
d|s|/ds is taken as sign(s) with sign(0) = 0.

Per element test function v, with w_q the quadrature weights:
  R_ck  += sum_q w_q [ (D_k grad c_k - c_k q_k).grad v - S_k v ]
  R_phi += sum_q w_q [ (sum_k a_k grad c_k + kappa grad phi).grad v - S_phi v ]
and face terms "Fv * v + G * dv/dn" collected per face point (see _face_res).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sps

from workload.configs import C_DIRICHLET, C_ELECTRODE, C_INFLOW, C_OUTFLOW

from .problem import Problem


def _z(shape):
    return np.zeros(shape)


class DG:
    def __init__(self, prob: Problem):
        self.P = prob
        msh = self.msh = prob.mesh
        self.m = prob.m
        self.N = self.m * msh.Nf
        self.xq = msh.vol_points()
        self.uq = prob.u(self.xq)                           # (E, Q, d)
        self.uhq = prob.uhat(self.xq)
        self.src = [prob.source(f, self.xq) for f in range(self.m)]
        # interior faces per axis
        self.iface = []
        for a in range(msh.dim):
            sel = msh.face_axis == a
            em, ep = msh.face_minus[sel], msh.face_plus[sel]
            pts = msh.face_points(em, a, 1)
            self.iface.append(dict(a=a, em=em, ep=ep, un=prob.u(pts)[..., a],
                                   uhn=prob.uhat(pts)[..., a]))
        # boundary faces per tag
        self.bface = []
        for t in range(2 * msh.dim):
            a, s = divmod(t, 2)
            side = -1 if s == 0 else 1
            el = msh.bfaces[t]
            pts = msh.face_points(el, a, side)
            d = dict(t=t, a=a, s=side, el=el, un=side * prob.u(pts)[..., a],
                     uhn=side * prob.uhat(pts)[..., a], cbc=prob.c_bc[t],
                     phid=prob.is_phi_dirichlet(t))
            if prob.c_bc[t] in (C_DIRICHLET, C_INFLOW):
                d["g"] = [None] + [prob.c_data(k, t) for k in range(1, self.m)]
            if d["phid"]:
                d["gphi"] = prob.phi_data(t)
            if prob.c_bc[t] == C_ELECTRODE:
                d["j0"], d["phiapp"] = prob.bv_data(t)
                d["prof"] = prob.j0_profile(pts)
            self.bface.append(d)

    # ------------------------------------------------------------------
    # interpolation helpers
    def fields(self, x):
        return np.asarray(x, float).reshape(self.m, self.msh.E, self.msh.nb)

    def _vol_state(self, X):
        msh = self.msh
        val = [X[f] @ msh.phi.T for f in range(self.m)]
        grad = [[X[f] @ msh.dphi[a].T for a in range(msh.dim)] for f in range(self.m)]
        return val, grad

    def _trace(self, X, elems, a, side, outward=False):
        msh = self.msh
        val = [X[f][elems] @ msh.fphi[(a, side)].T for f in range(self.m)]
        sgn = side if outward else 1.0
        dn = [sgn * (X[f][elems] @ msh.fdn[(a, side)].T) for f in range(self.m)]
        return val, dn

    # ------------------------------------------------------------------
    # pointwise fluxes: nonlinear (residual) and linearised
    def _vol_res(self, val, grad, f_src):
        P, d = self.P, self.msh.dim
        c = val
        gphi = grad[0]
        kap = sum(P.b[k - 1] * c[k] for k in range(1, self.m))
        vv = [-f_src[f] for f in range(self.m)]
        vg = [None] * self.m
        vg[0] = [sum(P.a[k - 1] * grad[k][i] for k in range(1, self.m)) + kap * gphi[i]
                 for i in range(d)]
        for k in range(1, self.m):
            q = [self.uq[..., i] - P.z[k - 1] * P.D[k - 1] * gphi[i] for i in range(d)]
            vg[k] = [P.D[k - 1] * grad[k][i] - c[k] * q[i] for i in range(d)]
        return vv, vg

    def _vol_lin(self, st, tr):
        """st = (val, grad) of the state with an optional trailing axis added;
        tr = dict(val, grad, du) of the perturbation (du: velocity perturbation)."""
        P, d = self.P, self.msh.dim
        c, grad = st
        dc, dgrad, du = tr["val"], tr["grad"], tr["du"]
        gphi, dgphi = grad[0], dgrad[0]
        kap = sum(P.b[k - 1] * c[k] for k in range(1, self.m))
        dkap = sum(P.b[k - 1] * dc[k] for k in range(1, self.m))
        vg = [None] * self.m
        vg[0] = [sum(P.a[k - 1] * dgrad[k][i] for k in range(1, self.m)) + dkap * gphi[i]
                 + kap * dgphi[i] for i in range(d)]
        for k in range(1, self.m):
            zD = P.z[k - 1] * P.D[k - 1]
            q = [self.uq_x[..., i] - zD * gphi[i] for i in range(d)]
            dq = [du[i] - zD * dgphi[i] for i in range(d)]
            vg[k] = [P.D[k - 1] * dgrad[k][i] - dc[k] * q[i] - c[k] * dq[i] for i in range(d)]
        return vg

    def _iface_res(self, vm, dm, vp, dp, un):
        """Interior face: returns Fv[f] (coefficient of v^- - v^+), Gm[f], Gp[f]
        (coefficients of dv^-/dn and dv^+/dn)."""
        P, dl = self.P, self.P.delta
        Fv, Gm, Gp = [None] * self.m, [None] * self.m, [None] * self.m
        kap_m = sum(P.b[k - 1] * vm[k] for k in range(1, self.m))
        kap_p = sum(P.b[k - 1] * vp[k] for k in range(1, self.m))
        jphi = vm[0] - vp[0]
        cur_m = sum(P.a[k - 1] * dm[k] for k in range(1, self.m)) + kap_m * dm[0]
        cur_p = sum(P.a[k - 1] * dp[k] for k in range(1, self.m)) + kap_p * dp[0]
        ajc = sum(P.a[k - 1] * (vm[k] - vp[k]) for k in range(1, self.m))
        Fv[0] = -0.5 * (cur_m + cur_p) + 0.5 * (kap_m + kap_p) * dl * jphi
        Gm[0] = -0.5 * ajc - 0.5 * kap_m * jphi
        Gp[0] = -0.5 * ajc - 0.5 * kap_p * jphi
        for k in range(1, self.m):
            D, zD = P.D[k - 1], P.z[k - 1] * P.D[k - 1]
            Qm = un - zD * dm[0]
            Qp = un - zD * dp[0]
            Qb = un - zD * 0.5 * (dm[0] + dp[0])
            jc = vm[k] - vp[k]
            Fv[k] = (-0.5 * D * (dm[k] + dp[k]) + D * dl * jc
                     + 0.5 * (vm[k] * Qm + vp[k] * Qp) + 0.5 * np.abs(Qb) * jc)
            Gm[k] = -0.5 * D * jc
            Gp[k] = -0.5 * D * jc
        return Fv, Gm, Gp

    def _iface_lin(self, st, tr, un):
        P, dl = self.P, self.P.delta
        vm, dm, vp, dp = st
        tvm, tdm, tvp, tdp, dun = tr["vm"], tr["dm"], tr["vp"], tr["dp"], tr["dun"]
        Fv, Gm, Gp = [None] * self.m, [None] * self.m, [None] * self.m
        kap_m = sum(P.b[k - 1] * vm[k] for k in range(1, self.m))
        kap_p = sum(P.b[k - 1] * vp[k] for k in range(1, self.m))
        dkap_m = sum(P.b[k - 1] * tvm[k] for k in range(1, self.m))
        dkap_p = sum(P.b[k - 1] * tvp[k] for k in range(1, self.m))
        jphi = vm[0] - vp[0]
        djphi = tvm[0] - tvp[0]
        dcur_m = (sum(P.a[k - 1] * tdm[k] for k in range(1, self.m)) + dkap_m * dm[0]
                  + kap_m * tdm[0])
        dcur_p = (sum(P.a[k - 1] * tdp[k] for k in range(1, self.m)) + dkap_p * dp[0]
                  + kap_p * tdp[0])
        dajc = sum(P.a[k - 1] * (tvm[k] - tvp[k]) for k in range(1, self.m))
        Fv[0] = (-0.5 * (dcur_m + dcur_p) + 0.5 * (dkap_m + dkap_p) * dl * jphi
                 + 0.5 * (kap_m + kap_p) * dl * djphi)
        Gm[0] = -0.5 * dajc - 0.5 * dkap_m * jphi - 0.5 * kap_m * djphi
        Gp[0] = -0.5 * dajc - 0.5 * dkap_p * jphi - 0.5 * kap_p * djphi
        for k in range(1, self.m):
            D, zD = P.D[k - 1], P.z[k - 1] * P.D[k - 1]
            Qm = un - zD * dm[0]
            Qp = un - zD * dp[0]
            Qb = un - zD * 0.5 * (dm[0] + dp[0])
            dQm = dun - zD * tdm[0]
            dQp = dun - zD * tdp[0]
            dQb = 0.5 * (dQm + dQp)
            jc = vm[k] - vp[k]
            djc = tvm[k] - tvp[k]
            Fv[k] = (-0.5 * D * (tdm[k] + tdp[k]) + D * dl * djc
                     + 0.5 * (tvm[k] * Qm + vm[k] * dQm + tvp[k] * Qp + vp[k] * dQp)
                     + 0.5 * np.sign(Qb) * dQb * jc + 0.5 * np.abs(Qb) * djc)
            Gm[k] = -0.5 * D * djc
            Gp[k] = -0.5 * D * djc
        return Fv, Gm, Gp

    # ------------------------------------------------------------------
    # Butler-Volmer electrode rate (Eqs. electrode, bv; Sec. 2.3)
    def _bv_conc(self, val):
        """Concentration of the reacting ion from the field traces."""
        P = self.P
        r = P.bv_ion
        if r < self.m:
            return val[r]
        return -sum(P.z[k - 1] * val[k] for k in range(1, self.m)) / P.z[self.m - 1]

    def _bv(self, bf, val):
        """g and its derivatives with respect to phi, c_r, J0 and phi_app."""
        P = self.P
        aa, ac = P.bv_alpha
        j0, pa = bf["j0"], bf["phiapp"]
        eta = pa - val[0]
        ea, ec = np.exp(aa * eta), np.exp(-ac * eta)
        c = self._bv_conc(val)
        g = j0 * (ea - c * ec)
        dphi = j0 * (-aa * ea - c * ac * ec)
        return g, dphi, -j0 * ec, ea - c * ec, -dphi

    def _bv_apply(self, Fv, rate):
        """Adds the electrode terms of the rate g to the value coefficients."""
        P = self.P
        r = P.bv_ion
        if r < self.m:
            Fv[r] = Fv[r] - rate
        Fv[0] = Fv[0] - P.z[r - 1] * rate

    def _bface_res(self, bf, val, dn):
        """Boundary face with outward normal derivative dn: returns Fv[f], G[f]."""
        P, dl = self.P, self.P.delta
        Fv = [0.0] * self.m
        G = [0.0] * self.m
        un = bf["un"]
        kap = sum(P.b[k - 1] * val[k] for k in range(1, self.m))
        for k in range(1, self.m):
            D, zD = P.D[k - 1], P.z[k - 1] * P.D[k - 1]
            Q = un - zD * dn[0]
            if bf["cbc"] == C_DIRICHLET:
                g = bf["g"][k]
                Fv[k] = (-D * dn[k] + D * dl * (val[k] - g) + np.maximum(Q, 0.0) * val[k]
                         + np.minimum(Q, 0.0) * g)
                G[k] = -D * (val[k] - g)
                G[0] = G[0] - P.a[k - 1] * (val[k] - g)
            elif bf["cbc"] == C_INFLOW:
                Fv[k] = un * bf["g"][k]
            elif bf["cbc"] == C_OUTFLOW:
                Fv[k] = Q * val[k]
        if bf["phid"]:
            gp = bf["gphi"]
            cur = sum(P.a[k - 1] * dn[k] for k in range(1, self.m)) + kap * dn[0]
            Fv[0] = -cur + kap * dl * (val[0] - gp)
            G[0] = G[0] - kap * (val[0] - gp)
        if bf["cbc"] == C_ELECTRODE:
            self._bv_apply(Fv, self._bv(bf, val)[0])
        return Fv, G

    def _bface_lin(self, bf, st, tr):
        P, dl = self.P, self.P.delta
        val, dn = st
        tv, tdn, dun, dg = tr["val"], tr["dn"], tr["dun"], tr["dg"]
        Fv = [0.0] * self.m
        G = [0.0] * self.m
        un = bf["un"]
        kap = sum(P.b[k - 1] * val[k] for k in range(1, self.m))
        dkap = sum(P.b[k - 1] * tv[k] for k in range(1, self.m))
        for k in range(1, self.m):
            D, zD = P.D[k - 1], P.z[k - 1] * P.D[k - 1]
            Q = un - zD * dn[0]
            dQ = dun - zD * tdn[0]
            if bf["cbc"] == C_DIRICHLET:
                g = bf["g"][k]
                sg = np.sign(Q)
                Fv[k] = (-D * tdn[k] + D * dl * (tv[k] - dg[k]) + np.maximum(Q, 0.0) * tv[k]
                         + 0.5 * (1.0 + sg) * dQ * val[k] + 0.5 * (1.0 - sg) * dQ * g
                         + np.minimum(Q, 0.0) * dg[k])
                G[k] = -D * (tv[k] - dg[k])
                G[0] = G[0] - P.a[k - 1] * (tv[k] - dg[k])
            elif bf["cbc"] == C_INFLOW:
                Fv[k] = dun * bf["g"][k] + un * dg[k]
            elif bf["cbc"] == C_OUTFLOW:
                Fv[k] = dQ * val[k] + Q * tv[k]
        if bf["phid"]:
            gp = bf["gphi"]
            dcur = (sum(P.a[k - 1] * tdn[k] for k in range(1, self.m)) + dkap * dn[0]
                    + kap * tdn[0])
            Fv[0] = -dcur + dkap * dl * (val[0] - gp) + kap * dl * tv[0]
            G[0] = G[0] - dkap * (val[0] - gp) - kap * tv[0]
        if bf["cbc"] == C_ELECTRODE:
            _, g_phi, g_c, g_j0, g_pa = self._bv(bf, val)
            rate = g_phi * tv[0] + g_c * self._bv_conc(tv)
            rate = rate + g_j0 * tr.get("dj0", 0.0) + g_pa * tr.get("dphiapp", 0.0)
            self._bv_apply(Fv, rate)
        return Fv, G

    # ------------------------------------------------------------------
    # residual
    def residual(self, x):
        msh = self.msh
        X = self.fields(x)
        R = np.zeros((self.m, msh.E, msh.nb))
        val, grad = self._vol_state(X)
        vv, vg = self._vol_res(val, grad, self.src)
        W = msh.wvol
        for f in range(self.m):
            R[f] += (vv[f] * W) @ msh.phi
            for i in range(msh.dim):
                R[f] += (vg[f][i] * W) @ msh.dphi[i]
        for fc in self.iface:
            a, em, ep = fc["a"], fc["em"], fc["ep"]
            vm, dm = self._trace(X, em, a, 1)
            vp, dp = self._trace(X, ep, a, -1)
            Fv, Gm, Gp = self._iface_res(vm, dm, vp, dp, fc["un"])
            w = msh.fw[a]
            for f in range(self.m):
                R[f][em] += (Fv[f] * w) @ msh.fphi[(a, 1)] + (Gm[f] * w) @ msh.fdn[(a, 1)]
                R[f][ep] += (-Fv[f] * w) @ msh.fphi[(a, -1)] + (Gp[f] * w) @ msh.fdn[(a, -1)]
        for bf in self.bface:
            a, s, el = bf["a"], bf["s"], bf["el"]
            val_b, dn_b = self._trace(X, el, a, s, outward=True)
            Fv, G = self._bface_res(bf, val_b, dn_b)
            w = msh.fw[a]
            for f in range(self.m):
                shp = (len(el), len(w))
                R[f][el] += ((np.broadcast_to(Fv[f], shp) * w) @ msh.fphi[(a, s)]
                             + (np.broadcast_to(G[f], shp) * w) @ (s * msh.fdn[(a, s)]))
        return R.reshape(-1)

    # ------------------------------------------------------------------
    # linearisation applied to a vector (matrix-free) -- also d/dPe and d/dg
    def lin_apply(self, x, v=None, du_scale=0.0, dg=None):
        """J(x) v + du_scale * dR/dPe(x) + dR/dg(x) dg, all exact."""
        msh, d = self.msh, self.msh.dim
        X = self.fields(x)
        Vv = self.fields(np.zeros(self.N) if v is None else v)
        Y = np.zeros((self.m, msh.E, msh.nb))
        self.uq_x = self.uq
        st = self._vol_state(X)
        tv = self._vol_state(Vv)
        tr = dict(val=tv[0], grad=tv[1], du=[du_scale * self.uhq[..., i] for i in range(d)])
        vg = self._vol_lin(st, tr)
        W = msh.wvol
        for f in range(self.m):
            for i in range(d):
                Y[f] += (vg[f][i] * W) @ msh.dphi[i]
        for fc in self.iface:
            a, em, ep = fc["a"], fc["em"], fc["ep"]
            s_m = self._trace(X, em, a, 1)
            s_p = self._trace(X, ep, a, -1)
            t_m = self._trace(Vv, em, a, 1)
            t_p = self._trace(Vv, ep, a, -1)
            tr = dict(vm=t_m[0], dm=t_m[1], vp=t_p[0], dp=t_p[1], dun=du_scale * fc["uhn"])
            Fv, Gm, Gp = self._iface_lin((s_m[0], s_m[1], s_p[0], s_p[1]), tr, fc["un"])
            w = msh.fw[a]
            for f in range(self.m):
                Y[f][em] += (Fv[f] * w) @ msh.fphi[(a, 1)] + (Gm[f] * w) @ msh.fdn[(a, 1)]
                Y[f][ep] += (-Fv[f] * w) @ msh.fphi[(a, -1)] + (Gp[f] * w) @ msh.fdn[(a, -1)]
        for bf in self.bface:
            a, s, el = bf["a"], bf["s"], bf["el"]
            st_b = self._trace(X, el, a, s, outward=True)
            tv_b = self._trace(Vv, el, a, s, outward=True)
            nqf = len(msh.fw[a])
            dgb = [0.0] * self.m
            if dg is not None and "g" in bf:
                nfn = msh.nn ** (d - 1)
                off = self.P.bnode_off[bf["t"]]
                for k in range(1, self.m):
                    gk = dg[k - 1, off: off + len(el) * nfn].reshape(len(el), nfn)
                    dgb[k] = gk @ msh.fpsi[a].T
            tr = dict(val=tv_b[0], dn=tv_b[1], dun=du_scale * bf["uhn"], dg=dgb)
            Fv, G = self._bface_lin(bf, st_b, tr)
            w = msh.fw[a]
            for f in range(self.m):
                shp = (len(el), nqf)
                Y[f][el] += ((np.broadcast_to(Fv[f], shp) * w) @ msh.fphi[(a, s)]
                             + (np.broadcast_to(G[f], shp) * w) @ (s * msh.fdn[(a, s)]))
        return Y.reshape(-1)

    def jac_apply(self, x, v):
        return self.lin_apply(x, v)

    def dR_dPe(self, x):
        return self.lin_apply(x, None, du_scale=1.0)

    # ------------------------------------------------------------------
    # sparse assembly of the exact Jacobian (linearisation applied to basis functions)
    def jacobian(self, x, fields=None):
        """Assembled J(x) as CSR.  `fields` optionally restricts to a list of
        (test field, trial field) pairs (e.g. the diagonal blocks)."""
        msh, d, m = self.msh, self.msh.dim, self.m
        X = self.fields(x)
        Nf, nb, E = msh.Nf, msh.nb, msh.E
        pairs = fields if fields is not None else [(f, g) for f in range(m) for g in range(m)]
        rows, cols, vals = [], [], []
        self.uq_x = self.uq[:, :, None, :]
        val, grad = self._vol_state(X)
        st = ([v[..., None] for v in val], [[gi[..., None] for gi in g] for g in grad])
        W = msh.wvol

        def add_block(f, g, er, ec, B):
            if not np.any(B):
                return
            r = (f * Nf + er[:, None] * nb + np.arange(nb)[None, :])
            c = (g * Nf + ec[:, None] * nb + np.arange(nb)[None, :])
            rows.append(np.broadcast_to(r[:, :, None], B.shape).reshape(-1))
            cols.append(np.broadcast_to(c[:, None, :], B.shape).reshape(-1))
            vals.append(B.reshape(-1))

        zero_q = 0.0
        for g in range(m):
            tval = [zero_q] * m
            tgrad = [[zero_q] * d for _ in range(m)]
            tval[g] = msh.phi[None]
            tgrad[g] = [msh.dphi[i][None] for i in range(d)]
            tr = dict(val=tval, grad=tgrad, du=[0.0] * d)
            vg = self._vol_lin(st, tr)
            for f in range(m):
                if (f, g) not in pairs:
                    continue
                B = np.zeros((E, nb, nb))
                for i in range(d):
                    coef = np.broadcast_to(vg[f][i], (E, W.shape[0], nb))
                    B += np.einsum("eqj,qi->eij", coef * W[None, :, None], msh.dphi[i])
                add_block(f, g, np.arange(E), np.arange(E), B)
        self.uq_x = self.uq
        for fc in self.iface:
            a, em, ep, un = fc["a"], fc["em"], fc["ep"], fc["un"]
            w = msh.fw[a]
            s_m = self._trace(X, em, a, 1)
            s_p = self._trace(X, ep, a, -1)
            st_f = tuple([v[..., None] for v in arr] for arr in (s_m[0], s_m[1], s_p[0], s_p[1]))
            unx = un[..., None]
            for g in range(m):
                for side in (1, -1):       # trial function on the "-" element (side 1) or "+"
                    z = [0.0] * m
                    tb_v = list(z)
                    tb_d = list(z)
                    tb_v[g] = msh.fphi[(a, side)][None]
                    tb_d[g] = msh.fdn[(a, side)][None]
                    if side == 1:
                        tr = dict(vm=tb_v, dm=tb_d, vp=list(z), dp=list(z), dun=0.0)
                        ecol = em
                    else:
                        tr = dict(vm=list(z), dm=list(z), vp=tb_v, dp=tb_d, dun=0.0)
                        ecol = ep
                    Fv, Gm, Gp = self._iface_lin(st_f, tr, unx)
                    for f in range(m):
                        if (f, g) not in pairs:
                            continue
                        shp = (len(em), len(w), nb)
                        Fb = np.broadcast_to(Fv[f], shp) * w[None, :, None]
                        Bm = (np.einsum("eqj,qi->eij", Fb, msh.fphi[(a, 1)])
                              + np.einsum("eqj,qi->eij", np.broadcast_to(Gm[f], shp) * w[None, :, None],
                                          msh.fdn[(a, 1)]))
                        Bp = (np.einsum("eqj,qi->eij", -Fb, msh.fphi[(a, -1)])
                              + np.einsum("eqj,qi->eij", np.broadcast_to(Gp[f], shp) * w[None, :, None],
                                          msh.fdn[(a, -1)]))
                        add_block(f, g, em, ecol, Bm)
                        add_block(f, g, ep, ecol, Bp)
        for bf in self.bface:
            a, s, el = bf["a"], bf["s"], bf["el"]
            w = msh.fw[a]
            st_b = self._trace(X, el, a, s, outward=True)
            st_bx = ([v[..., None] for v in st_b[0]], [v[..., None] for v in st_b[1]])
            bfx = dict(bf)
            bfx["un"] = bf["un"][..., None]
            if "g" in bf:
                bfx["g"] = [None] + [gk[..., None] for gk in bf["g"][1:]]
            if "gphi" in bf:
                bfx["gphi"] = bf["gphi"][..., None]
            for key in ("j0", "phiapp"):
                if key in bf:
                    bfx[key] = bf[key][..., None]
            for g in range(m):
                tb_v = [0.0] * m
                tb_d = [0.0] * m
                tb_v[g] = msh.fphi[(a, s)][None]
                tb_d[g] = s * msh.fdn[(a, s)][None]
                tr = dict(val=tb_v, dn=tb_d, dun=0.0, dg=[0.0] * m)
                Fv, G = self._bface_lin(bfx, st_bx, tr)
                for f in range(m):
                    if (f, g) not in pairs:
                        continue
                    shp = (len(el), len(w), nb)
                    B = (np.einsum("eqj,qi->eij", np.broadcast_to(Fv[f], shp) * w[None, :, None],
                                   msh.fphi[(a, s)])
                         + np.einsum("eqj,qi->eij", np.broadcast_to(G[f], shp) * w[None, :, None],
                                     s * msh.fdn[(a, s)]))
                    add_block(f, g, el, el, B)
        rows = np.concatenate(rows)
        cols = np.concatenate(cols)
        vals = np.concatenate(vals)
        return sps.csr_matrix((vals, (rows, cols)), shape=(self.N, self.N))

    def dR_dg(self, x):
        """dR/d(boundary nodal data) as a dense (N, (m-1)*n_bnode) array built from
        unit perturbations of the data (exact: R is affine in the data)."""
        nbn = self.P.n_bnode
        out = np.zeros((self.N, (self.m - 1) * nbn))
        for k in range(self.m - 1):
            for j in range(nbn):
                dg = np.zeros((self.m - 1, nbn))
                dg[k, j] = 1.0
                out[:, k * nbn + j] = self.lin_apply(x, None, dg=dg)
        return out

    def dR_dg_T(self, x, lam):
        """lam^T dR/dg without forming the matrix: one face pass per data node."""
        nbn = self.P.n_bnode
        res = np.zeros((self.m - 1, nbn))
        msh, d = self.msh, self.msh.dim
        X = self.fields(x)
        L = self.fields(lam)
        nfn = msh.nn ** (d - 1)
        for bf in self.bface:
            if "g" not in bf:
                continue
            a, s, el = bf["a"], bf["s"], bf["el"]
            w = msh.fw[a]
            off = self.P.bnode_off[bf["t"]]
            st_b = self._trace(X, el, a, s, outward=True)
            st_bx = ([v[..., None] for v in st_b[0]], [v[..., None] for v in st_b[1]])
            bfx = dict(bf)
            bfx["un"] = bf["un"][..., None]
            bfx["g"] = [None] + [gk[..., None] for gk in bf["g"][1:]]
            if "gphi" in bf:
                bfx["gphi"] = bf["gphi"][..., None]
            lv, ldn = self._trace(L, el, a, s, outward=True)
            for k in range(1, self.m):
                dgb = [0.0] * self.m
                dgb[k] = msh.fpsi[a][None]                 # (1, nqf, nfn)
                tr = dict(val=[0.0] * self.m, dn=[0.0] * self.m, dun=0.0, dg=dgb)
                Fv, G = self._bface_lin(bfx, st_bx, tr)
                acc = 0.0
                for f in range(self.m):
                    shp = (len(el), len(w), nfn)
                    acc = acc + np.einsum("eqj,eq->ej", np.broadcast_to(Fv[f], shp) * w[None, :, None],
                                          lv[f])
                    acc = acc + np.einsum("eqj,eq->ej", np.broadcast_to(G[f], shp) * w[None, :, None],
                                          ldn[f])
                res[k - 1, off: off + len(el) * nfn] = np.asarray(acc).reshape(-1)
        return res

    def dR_dbv_T(self, x, lam):
        """(lam^T dR/dJ0_t, lam^T dR/dphi_app_t) for every box face t (zero on
        faces without an electrode); J0_t scales the face's exchange-current
        profile."""
        msh, d = self.msh, self.msh.dim
        X, L = self.fields(x), self.fields(lam)
        out_j0, out_pa = np.zeros(2 * d), np.zeros(2 * d)
        for bf in self.bface:
            if bf["cbc"] != C_ELECTRODE:
                continue
            a, s, el = bf["a"], bf["s"], bf["el"]
            w = msh.fw[a]
            st_b = self._trace(X, el, a, s, outward=True)
            lv, ldn = self._trace(L, el, a, s, outward=True)
            for which, key, pert in ((0, "dj0", bf["prof"]), (1, "dphiapp", np.ones_like(bf["prof"]))):
                tr = dict(val=[0.0] * self.m, dn=[0.0] * self.m, dun=0.0, dg=[0.0] * self.m)
                tr[key] = pert
                Fv, G = self._bface_lin(bf, st_b, tr)
                acc = sum(float(np.sum(np.broadcast_to(Fv[f], lv[f].shape) * w * lv[f])) for f in range(self.m))
                (out_j0 if which == 0 else out_pa)[bf["t"]] = acc
        return out_j0, out_pa

    def electrode_currents(self, x):
        """Integral of the reacting ion's rate g over each box face (zero where
        there is no electrode)."""
        msh, d = self.msh, self.msh.dim
        X = self.fields(x)
        out = np.zeros(2 * d)
        for bf in self.bface:
            if bf["cbc"] != C_ELECTRODE:
                continue
            val, _ = self._trace(X, bf["el"], bf["a"], bf["s"], outward=True)
            out[bf["t"]] = float(np.sum(self._bv(bf, val)[0] * msh.fw[bf["a"]]))
        return out

    # ------------------------------------------------------------------
    # objectives: 0 = outflow flux of species 1 through the x+ box face,
    # 1 = reaction rate of the reacting ion integrated over the first
    # electrode face (the cell current divided by its valence)
    def _electrode_face(self):
        for bf in self.bface:
            if bf["cbc"] == C_ELECTRODE:
                return bf
        raise ValueError("objective 1 needs an electrode face")

    def objective(self, x, kind=0):
        msh = self.msh
        X = self.fields(x)
        P = self.P
        if kind == 1:
            bf = self._electrode_face()
            val, _ = self._trace(X, bf["el"], bf["a"], bf["s"], outward=True)
            return float(np.sum(self._bv(bf, val)[0] * msh.fw[bf["a"]]))
        bf = self.bface[1]
        val, dn = self._trace(X, bf["el"], bf["a"], bf["s"], outward=True)
        Q = bf["un"] - P.z[0] * P.D[0] * dn[0]
        return float(np.sum((Q * val[1]) * msh.fw[bf["a"]]))

    def objective_grad(self, x, kind=0):
        """(dJ/dx, dJ/dPe) of the objective."""
        msh = self.msh
        P = self.P
        X = self.fields(x)
        g = np.zeros((self.m, msh.E, msh.nb))
        if kind == 1:
            bf = self._electrode_face()
            a, s, el = bf["a"], bf["s"], bf["el"]
            val, _ = self._trace(X, el, a, s, outward=True)
            _, g_phi, g_c, _, _ = self._bv(bf, val)
            w = msh.fw[a]
            g[0][el] += (g_phi * w) @ msh.fphi[(a, s)]
            r = P.bv_ion
            for k in range(1, self.m):
                dck = (1.0 if k == r else 0.0) if r < self.m else -P.z[k - 1] / P.z[self.m - 1]
                if dck != 0.0:
                    g[k][el] += (dck * g_c * w) @ msh.fphi[(a, s)]
            return g.reshape(-1), 0.0
        bf = self.bface[1]
        a, s, el = bf["a"], bf["s"], bf["el"]
        val, dn = self._trace(X, el, a, s, outward=True)
        zD = P.z[0] * P.D[0]
        Q = bf["un"] - zD * dn[0]
        w = msh.fw[a]
        g[1][el] += (Q * w) @ msh.fphi[(a, s)]
        g[0][el] += (-zD * val[1] * w) @ (s * msh.fdn[(a, s)])
        dPe = float(np.sum(bf["uhn"] * val[1] * w))
        return g.reshape(-1), dPe

    def objective_dbv(self, x, kind=0):
        """Explicit derivatives (dJ/dJ0_t, dJ/dphi_app_t) of the objective at fixed x."""
        d = self.msh.dim
        out_j0, out_pa = np.zeros(2 * d), np.zeros(2 * d)
        if kind == 1:
            bf = self._electrode_face()
            val, _ = self._trace(self.fields(x), bf["el"], bf["a"], bf["s"], outward=True)
            _, _, _, g_j0, g_pa = self._bv(bf, val)
            w = self.msh.fw[bf["a"]]
            out_j0[bf["t"]] = float(np.sum(g_j0 * bf["prof"] * w))
            out_pa[bf["t"]] = float(np.sum(g_pa * w))
        return out_j0, out_pa
