"""Geometric multigrid for one concentration block (test infrastructure: only
tests/ and the bench's CPU leg use it; the product path never imports it).

Sec. 4.1 approximates the inverse of each concentration block A_{c_k c_k} by
iterations preconditioned with an h-multigrid cycle whose smoother is the
same additive-Schwarz block ILU(0) used on its own by the first approach, and
whose coarsest grid is solved by a full LU factorisation (the solver listing of
Appendix A: Richardson smoothing on the levels, direct coarse solve).  On one
device the Schwarz decomposition has a single subdomain, so the smoother is
the block ILU(0) of the whole level.

Readings taken here (the paper fixes none of them):
  * levels: the structured box coarsened by 2 along every axis while every
    element count is even (down to a single element where the counts allow);
  * coarse operators: Galerkin products P^T A P.  The coarse space (degree-p
    polynomials on each coarse element) lies inside the fine one, and P
    evaluates a coarse element's polynomial at the nodes of its 2^d children;
  * smoother: nu steps x <- x + M^{-1} (b - A x) before and after the coarse
    correction, M the block ILU(0) of the level in the lexicographic element
    order (M = (D + L) D^{-1} (D + U) with L, U the strictly lower / upper
    blocks of A and D_i = A_ii - sum_{k lower} A_ik D_k^{-1} A_ki: on the
    7-point block pattern every other fill position lies outside the pattern);
  * one V-cycle per concentration block and preconditioner application.

Everything is written from those definitions: scipy sparse products for P and
the Galerkin operators, dense numpy blocks for the ILU(0), numpy's dense LU
for the coarsest level.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .mesh import _kron_list
from .quadrature import gll_points, lagrange


def child_prolongations(p: int, dim: int):
    """Pi[c] (nb x nb): Pi[c][j, i] = value of coarse basis function i at fine
    node j of child c; child c has bit a of c set when it is the upper half of
    the coarse element along axis a (axis 0 fastest in the node numbering)."""
    xn = gll_points(p)
    half = {}
    for s in (0, 1):
        # child s covers [-1, 0] (s = 0) or [0, 1] (s = 1) of the parent's reference interval
        V, _ = lagrange(xn, (xn + (2 * s - 1)) / 2.0)
        half[s] = V
    return [_kron_list([half[(c >> a) & 1] for a in range(dim)]) for c in range(2 ** dim)]


def neighbours(n):
    """Slot-ordered neighbours (-x, +x, -y, +y, -z, +z), -1 on the boundary, of
    the lexicographic elements of an n[0] x ... grid."""
    dim = len(n)
    E = int(np.prod(n))
    stride = [int(np.prod(n[:a])) for a in range(dim)]
    e = np.arange(E)
    idx = np.stack([(e // stride[a]) % n[a] for a in range(dim)], axis=1)
    nbr = np.full((E, 2 * dim), -1, dtype=np.int64)
    for a in range(dim):
        nbr[idx[:, a] > 0, 2 * a] = e[idx[:, a] > 0] - stride[a]
        nbr[idx[:, a] < n[a] - 1, 2 * a + 1] = e[idx[:, a] < n[a] - 1] + stride[a]
    return nbr


def prolongation(nf, p: int):
    """Sparse P from the coarse grid nf // 2 to the fine grid nf (both with one
    field's nodal DOFs, element-major)."""
    dim = len(nf)
    nc = [v // 2 for v in nf]
    nb = (p + 1) ** dim
    Pi = child_prolongations(p, dim)
    Ef = int(np.prod(nf))
    rows, cols, vals = [], [], []
    sf = [int(np.prod(nf[:a])) for a in range(dim)]
    sc = [int(np.prod(nc[:a])) for a in range(dim)]
    jj, ii = np.meshgrid(np.arange(nb), np.arange(nb), indexing="ij")
    for e in range(Ef):
        idx = [(e // sf[a]) % nf[a] for a in range(dim)]
        parent = sum((idx[a] // 2) * sc[a] for a in range(dim))
        child = sum((idx[a] % 2) << a for a in range(dim))
        rows.append(e * nb + jj.reshape(-1))
        cols.append(parent * nb + ii.reshape(-1))
        vals.append(Pi[child].reshape(-1))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(Ef * nb, int(np.prod(nc)) * nb))


class BlockILU0:
    """Block ILU(0) of a block-sparse matrix on the element graph `nbr`, in the
    lexicographic element order (see the module notes)."""

    def __init__(self, A, nbr, nb):
        A = sp.csr_matrix(A)
        self.E = nbr.shape[0]
        self.nb = nb
        self.nbr = nbr

        def blk(i, j):
            return A[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb].toarray()

        self.A = {}
        for i in range(self.E):
            self.A[(i, i)] = blk(i, i)
            for j in nbr[i]:
                if j >= 0:
                    self.A[(i, int(j))] = blk(i, int(j))
        self.D = [None] * self.E
        self.Dinv = [None] * self.E
        for i in range(self.E):
            Di = self.A[(i, i)].copy()
            for k in nbr[i]:
                if 0 <= k < i:
                    Di -= self.A[(i, int(k))] @ self.Dinv[int(k)] @ self.A[(int(k), i)]
            self.D[i] = Di
            self.Dinv[i] = np.linalg.inv(Di)

    def _lower(self, i):
        return [int(k) for k in self.nbr[i] if 0 <= k < i]

    def _upper(self, i):
        return [int(k) for k in self.nbr[i] if k > i]

    def solve(self, r):
        """M^{-1} r: (D + L) w = r, then (I + D^{-1} U) z = w."""
        nb = self.nb
        R = np.asarray(r, float).reshape(self.E, nb)
        w = np.zeros_like(R)
        for i in range(self.E):
            t = R[i].copy()
            for k in self._lower(i):
                t -= self.A[(i, k)] @ w[k]
            w[i] = self.Dinv[i] @ t
        z = np.zeros_like(R)
        for i in reversed(range(self.E)):
            t = np.zeros(nb)
            for k in self._upper(i):
                t += self.A[(i, k)] @ z[k]
            z[i] = w[i] - self.Dinv[i] @ t
        return z.reshape(-1)

    def solve_T(self, r):
        """M^{-T} r with M^T = (D + U)^T D^{-T} (D + L)^T."""
        nb = self.nb
        R = np.asarray(r, float).reshape(self.E, nb)
        y = np.zeros_like(R)
        for i in range(self.E):  # (D + U)^T y = r: block i is coupled to U_ki^T = A_ki^T, k < i
            t = R[i].copy()
            for k in self._lower(i):
                t -= self.A[(k, i)].T @ y[k]
            y[i] = np.linalg.solve(self.D[i].T, t)
        y = np.stack([self.D[i].T @ y[i] for i in range(self.E)])
        z = np.zeros_like(R)
        for i in reversed(range(self.E)):  # (D + L)^T z = y: coupled to L_ki^T = A_ki^T, k > i
            t = y[i].copy()
            for k in self._upper(i):
                t -= self.A[(k, i)].T @ z[k]
            z[i] = np.linalg.solve(self.D[i].T, t)
        return z.reshape(-1)

    def matrix(self):
        """M = (D + L) D^{-1} (D + U) as a dense matrix (small cases)."""
        nb, E = self.nb, self.E
        DL = np.zeros((E * nb, E * nb))
        DU = np.zeros((E * nb, E * nb))
        Dinv = np.zeros((E * nb, E * nb))
        for i in range(E):
            s = slice(i * nb, (i + 1) * nb)
            DL[s, s] = self.D[i]
            DU[s, s] = self.D[i]
            Dinv[s, s] = self.Dinv[i]
            for k in self._lower(i):
                DL[s, k * nb:(k + 1) * nb] = self.A[(i, k)]
            for k in self._upper(i):
                DU[s, k * nb:(k + 1) * nb] = self.A[(i, k)]
        return DL @ Dinv @ DU


def coarsen_dims(n, max_elems=None):
    """Element counts of the levels, finest first (see the module notes);
    max_elems: stop at the first level with at most that many elements."""
    stop = 1 if max_elems is None else max_elems
    dims = [tuple(int(v) for v in n)]
    while all(v % 2 == 0 for v in dims[-1]) and int(np.prod(dims[-1])) > stop:
        dims.append(tuple(v // 2 for v in dims[-1]))
    return dims


class GMG:
    """V-cycle for one concentration block A (N_f x N_f, element-major nodal
    DOFs) on the structured grid n with order p."""

    def __init__(self, A, n, p, nu=2, max_elems=None):
        self.p = p
        self.nu = nu
        self.dim = len(n)
        self.nb = (p + 1) ** self.dim
        self.dims = coarsen_dims(n, max_elems)
        self.A = [sp.csr_matrix(A)]
        self.P = []
        for l in range(len(self.dims) - 1):
            P = prolongation(self.dims[l], p)
            self.P.append(P)
            self.A.append(sp.csr_matrix(P.T @ self.A[l] @ P))
        self.ilu = [BlockILU0(self.A[l], neighbours(self.dims[l]), self.nb) for l in range(len(self.dims) - 1)]
        self.coarse = self.A[-1].toarray()

    @property
    def levels(self):
        return len(self.dims)

    def _smooth(self, l, b, x, transpose):
        A = self.A[l].T if transpose else self.A[l]
        Minv = self.ilu[l].solve_T if transpose else self.ilu[l].solve
        for _ in range(self.nu):
            x = x + Minv(b - A @ x)
        return x

    def vcycle(self, b, l=0, transpose=False):
        """One V-cycle from a zero initial guess (transpose: the cycle of A^T
        with the transposed smoother, which is the exact transpose)."""
        if l == self.levels - 1:
            return np.linalg.solve(self.coarse.T if transpose else self.coarse, b)
        A = self.A[l].T if transpose else self.A[l]
        x = self._smooth(l, b, np.zeros_like(b), transpose)
        rc = self.P[l].T @ (b - A @ x)
        x = x + self.P[l] @ self.vcycle(rc, l + 1, transpose)
        return self._smooth(l, b, x, transpose)
