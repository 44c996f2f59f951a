"""Structured box mesh, DOF indexing and full tensor tabulations (test infrastructure).

Indexing (the paper gives only the block order [phi; c_1; ...; c_{m-1}]):
  element e = ix + nx*(iy + ny*iz); local node l = a + (p+1)*(b + (p+1)*c)
  (a along x); global DOF = f*N_f + e*n_b + l with field f = 0 for phi and
  f = k for c_k.  Interior faces: all x-normal faces first, ordered by their
  lower ("-") element, then y, then z; the face normal points from "-" to "+".
  Boundary faces: grouped by box-face tag 0..5 (x-, x+, y-, y+, z-, z+), each
  group ordered by element index.
"""
from __future__ import annotations

from functools import reduce

import numpy as np

from .quadrature import gauss_legendre, gll_points, lagrange


def _kron_list(mats):
    """kron(M_{d-1}, ..., M_0): the first listed (axis 0) index runs fastest."""
    return reduce(lambda acc, M: np.kron(M, acc), mats[1:], mats[0])


class BoxMesh:
    def __init__(self, dim, n, lo, hi, p, nq=None):
        self.dim = dim
        self.n = tuple(int(v) for v in n[:dim])
        self.lo = np.array(lo[:dim], float)
        self.hi = np.array(hi[:dim], float)
        self.p = p
        self.nn = p + 1                         # nodes per axis
        self.nq = p + 2 if nq is None else nq   # Gauss points per axis
        self.nb = self.nn ** dim
        self.E = int(np.prod(self.n))
        self.h = (self.hi - self.lo) / np.array(self.n, float)
        self.Nf = self.E * self.nb
        strides = [1]
        for a in range(1, dim):
            strides.append(strides[-1] * self.n[a - 1])
        self.stride = strides
        e = np.arange(self.E)
        self.eidx = np.stack([(e // strides[a]) % self.n[a] for a in range(dim)], axis=1)
        # neighbours in slot order (-x, +x, -y, +y, -z, +z); -1 on the boundary
        nbr = np.full((self.E, 2 * dim), -1, dtype=np.int64)
        for a in range(dim):
            lo_ok = self.eidx[:, a] > 0
            hi_ok = self.eidx[:, a] < self.n[a] - 1
            nbr[lo_ok, 2 * a] = e[lo_ok] - strides[a]
            nbr[hi_ok, 2 * a + 1] = e[hi_ok] + strides[a]
        self.nbr = nbr
        fm, fp, fa = [], [], []
        for a in range(dim):
            sel = e[self.eidx[:, a] < self.n[a] - 1]
            fm.append(sel)
            fp.append(sel + strides[a])
            fa.append(np.full(len(sel), a))
        self.face_minus = np.concatenate(fm)
        self.face_plus = np.concatenate(fp)
        self.face_axis = np.concatenate(fa)
        self.bfaces = {}
        for t in range(2 * dim):
            a, s = divmod(t, 2)
            target = 0 if s == 0 else self.n[a] - 1
            self.bfaces[t] = e[self.eidx[:, a] == target]
        # reference tables
        self.xn = gll_points(p)
        self.xq, self.wq = gauss_legendre(self.nq)
        self.V, self.Dq = lagrange(self.xn, self.xq)             # (nq, nn)
        self.Vend = {s: lagrange(self.xn, [float(s)])[0] for s in (-1, 1)}
        self.Dend = {s: lagrange(self.xn, [float(s)])[1] for s in (-1, 1)}
        self._tabulate()

    # ---- tabulations -------------------------------------------------
    def _tabulate(self):
        d = self.dim
        V, Dq = self.V, self.Dq
        self.phi = _kron_list([V] * d)                          # (Q, nb)
        self.dphi = []
        for a in range(d):
            mats = [Dq * (2.0 / self.h[b]) if b == a else V for b in range(d)]
            self.dphi.append(_kron_list(mats))
        self.wvol = _kron_list([self.wq[:, None]] * d)[:, 0] * np.prod(self.h / 2.0)
        # face tabulations: (axis, side) -> value and d/dx_axis at face points
        self.fphi, self.fdn, self.fw, self.fnodes, self.fpsi = {}, {}, {}, {}, {}
        for a in range(d):
            tang = [b for b in range(d) if b != a]
            wf = np.ones(1)
            for b in tang:
                wf = np.kron(self.wq, wf)
            jac = np.prod([self.h[b] / 2.0 for b in tang]) if tang else 1.0
            self.fw[a] = wf * jac
            for s in (-1, 1):
                mats = [self.Vend[s] if b == a else V for b in range(d)]
                self.fphi[(a, s)] = _kron_list(mats)
                mats = [self.Dend[s] * (2.0 / self.h[a]) if b == a else V for b in range(d)]
                self.fdn[(a, s)] = _kron_list(mats)
                # local indices of the face nodes, tangential lower axis fastest
                sel = [np.array([0 if s < 0 else self.p]) if b == a else np.arange(self.nn)
                       for b in range(d)]
                grid = np.meshgrid(*sel, indexing="ij")
                lidx = sum(grid[b] * self.nn ** b for b in range(d))
                # order so that axis 0 is fastest: transpose the meshgrid result
                lidx = np.transpose(lidx, axes=list(range(d))[::-1]).reshape(-1)
                self.fnodes[(a, s)] = lidx
            # Lagrange basis of the face nodes at the face points (tangential tensor)
            self.fpsi[a] = _kron_list([V] * len(tang)) if tang else np.ones((1, 1))

    # ---- geometry ----------------------------------------------------
    def elem_lo(self, e):
        return self.lo + self.eidx[e] * self.h

    def vol_points(self):
        """Physical coordinates of the volume Gauss points, (E, Q, d)."""
        d = self.dim
        ref = [(self.xq + 1.0) / 2.0] * d
        grids = np.meshgrid(*ref, indexing="ij")            # axis0 first
        pts = np.stack([np.transpose(g, list(range(d))[::-1]).reshape(-1) for g in grids], axis=1)
        lo = self.lo + self.eidx * self.h                    # (E, d)
        return lo[:, None, :] + pts[None, :, :] * self.h[None, None, :]

    def face_points(self, elems, a, s):
        """Physical coordinates of the Gauss points of face (axis a, side s) of elems."""
        d = self.dim
        tang = [b for b in range(d) if b != a]
        ref = [(self.xq + 1.0) / 2.0] * len(tang)
        if tang:
            grids = np.meshgrid(*ref, indexing="ij")
            pts_t = np.stack([np.transpose(g, list(range(len(tang)))[::-1]).reshape(-1)
                              for g in grids], axis=1)
        else:
            pts_t = np.zeros((1, 0))
        nqf = pts_t.shape[0]
        pts = np.zeros((nqf, d))
        for i, b in enumerate(tang):
            pts[:, b] = pts_t[:, i]
        pts[:, a] = 0.0 if s < 0 else 1.0
        lo = self.lo + self.eidx[elems] * self.h
        return lo[:, None, :] + pts[None, :, :] * self.h[None, None, :]

    def node_points(self):
        """Physical coordinates of all nodes, (E, nb, d)."""
        d = self.dim
        ref = [(self.xn + 1.0) / 2.0] * d
        grids = np.meshgrid(*ref, indexing="ij")
        pts = np.stack([np.transpose(g, list(range(d))[::-1]).reshape(-1) for g in grids], axis=1)
        lo = self.lo + self.eidx * self.h
        return lo[:, None, :] + pts[None, :, :] * self.h[None, None, :]

    @property
    def diameter(self):
        """Cell diameter (length of the element diagonal)."""
        return float(np.sqrt(np.sum(self.h ** 2)))
