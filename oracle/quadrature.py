"""1-D reference rules on [-1, 1] (test infrastructure; see oracle/__init__).

The scheme uses tensor-product hexahedral elements and integrates with a
quadrature of higher order than the polynomial degree (Sec. 4 intro, no GLL
collocation).  Reading used here: nodal Lagrange basis on the p+1
Gauss-Lobatto-Legendre points, Gauss-Legendre quadrature with p+2 points.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as leg


def gauss_legendre(nq: int):
    """Gauss-Legendre points and weights (exact for degree <= 2 nq - 1)."""
    x, w = leg.leggauss(nq)
    return np.asarray(x, float), np.asarray(w, float)


def gll_points(p: int) -> np.ndarray:
    """Gauss-Lobatto-Legendre points: -1, the roots of P_p', +1."""
    if p < 1:
        raise ValueError("p >= 1 required")
    c = np.zeros(p + 1)
    c[p] = 1.0
    inner = leg.legroots(leg.legder(c)) if p >= 2 else np.zeros(0)
    return np.concatenate([[-1.0], np.sort(np.real(inner)), [1.0]])


def lagrange(nodes: np.ndarray, pts: np.ndarray):
    """Values V[q, j] = l_j(pts[q]) and derivatives Dv[q, j] = l_j'(pts[q]) of the
    Lagrange polynomials on `nodes`, by the product formula
        l_j(x)  = prod_{i != j} (x - x_i) / (x_j - x_i)
        l_j'(x) = sum_{k != j} 1/(x_j - x_k) prod_{i != j,k} (x - x_i)/(x_j - x_i).
    """
    nodes = np.asarray(nodes, float)
    pts = np.atleast_1d(np.asarray(pts, float))
    n = len(nodes)
    V = np.ones((len(pts), n))
    Dv = np.zeros((len(pts), n))
    for j in range(n):
        for i in range(n):
            if i != j:
                V[:, j] *= (pts - nodes[i]) / (nodes[j] - nodes[i])
        for k in range(n):
            if k == j:
                continue
            term = np.full(len(pts), 1.0 / (nodes[j] - nodes[k]))
            for i in range(n):
                if i != j and i != k:
                    term *= (pts - nodes[i]) / (nodes[j] - nodes[i])
            Dv[:, j] += term
    return V, Dv
