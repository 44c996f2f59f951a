"""Pins of the oracle's geometric multigrid for the concentration blocks
(oracle/mg.py; Sec. 4.1 GMG with the block ILU(0) smoother), against what the
definitions fix independently of the code:

* the nested prolongation reproduces every coarse polynomial of per-axis
  degree <= p at the fine nodes (values computed from the polynomial itself);
* the block ILU(0) factor M = (D + L) D^{-1} (D + U) equals A on every block
  of the 7-point (5-point) element pattern, the defining property of ILU(0),
  and its solves are M^{-1} and M^{-T};
* the two-level coarse-grid correction with the Galerkin operator is a
  projection (C^2 = C) with P^T A C = 0;
* the V-cycle's transpose is its adjoint, and on a diffusion-dominated block
  the cycle contracts the error with a factor that does not grow with 1/h;
* the level sequence of the structured coarsening.
"""
import numpy as np
import pytest

from oracle import mg
from oracle.dg import DG
from oracle.mesh import BoxMesh
from oracle.problem import Problem
from tests.oracle_cases import gmg_box
from workload import boundary_data, random_state


def _conc_block(cfg, k=1):
    dg = DG(Problem(cfg, boundary_data(cfg)))
    x = random_state(cfg)
    J = dg.jacobian(x, fields=[(k, k)]).tocsr()
    Nf = dg.msh.Nf
    return J[k * Nf:(k + 1) * Nf, k * Nf:(k + 1) * Nf], dg


@pytest.mark.parametrize("dim,p", [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2)])
def test_prolongation_reproduces_coarse_polynomials(dim, p):
    nc = (3, 2, 2)[:dim]
    nf = tuple(2 * v for v in nc)
    rng = np.random.default_rng(3)
    coef = rng.uniform(-1, 1, size=(p + 1,) * dim)

    def f(pts):
        out = np.zeros(len(pts))
        for idx in np.ndindex(*coef.shape):
            out += coef[idx] * np.prod([pts[:, a] ** idx[a] for a in range(dim)], axis=0)
        return out

    lo, hi = (0.0,) * dim, (1.0, 0.7, 0.4)[:dim]
    xc = BoxMesh(dim, nc, lo, hi, p).node_points().reshape(-1, dim)
    xf = BoxMesh(dim, nf, lo, hi, p).node_points().reshape(-1, dim)
    P = mg.prolongation(nf, p)
    assert np.abs(P @ f(xc) - f(xf)).max() <= 1e-12 * np.abs(f(xf)).max()
    # each fine node takes one coarse element's polynomial: rows sum to 1
    assert np.allclose(np.asarray(P.sum(axis=1)).ravel(), 1.0, atol=1e-13)


@pytest.mark.parametrize("dim,n,nb", [(2, (4, 3), 4), (3, (3, 2, 2), 8), (3, (2, 3, 2), 27)])
def test_block_ilu0_agrees_with_A_on_the_pattern(dim, n, nb):
    nbr = mg.neighbours(n)
    E = nbr.shape[0]
    rng = np.random.default_rng(11)
    A = np.zeros((E * nb, E * nb))
    for i in range(E):
        A[i * nb:(i + 1) * nb, i * nb:(i + 1) * nb] = rng.uniform(-1, 1, (nb, nb)) + 4 * nb * np.eye(nb)
        for j in nbr[i]:
            if j >= 0:
                A[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb] = rng.uniform(-1, 1, (nb, nb))
    ilu = mg.BlockILU0(A, nbr, nb)
    M = ilu.matrix()
    mask = np.zeros((E, E), bool)
    for i in range(E):
        mask[i, i] = True
        for j in nbr[i]:
            if j >= 0:
                mask[i, j] = True
    bm = np.kron(mask, np.ones((nb, nb), bool))
    assert np.abs((M - A)[bm]).max() <= 1e-12 * np.abs(A).max()
    assert np.abs((M - A)[~bm]).max() > 1e-6  # fill outside the pattern is dropped
    r = rng.uniform(-1, 1, E * nb)
    assert np.allclose(ilu.solve(r), np.linalg.solve(M, r), rtol=0, atol=1e-12 * np.abs(np.linalg.solve(M, r)).max())
    assert np.allclose(ilu.solve_T(r), np.linalg.solve(M.T, r), rtol=0,
                       atol=1e-12 * np.abs(np.linalg.solve(M.T, r)).max())


def test_level_sequence():
    assert mg.coarsen_dims((16, 16, 16)) == [(16, 16, 16), (8, 8, 8), (4, 4, 4), (2, 2, 2), (1, 1, 1)]
    assert mg.coarsen_dims((64, 16, 8)) == [(64, 16, 8), (32, 8, 4), (16, 4, 2), (8, 2, 1)]
    assert mg.coarsen_dims((6, 4)) == [(6, 4), (3, 2)]
    assert mg.coarsen_dims((4, 4)) == [(4, 4), (2, 2), (1, 1)]
    assert mg.coarsen_dims((4, 4), max_elems=4) == [(4, 4), (2, 2)]


@pytest.mark.parametrize("dim,p", [(2, 1), (3, 1), (2, 2)])
def test_coarse_grid_correction_is_a_projection(dim, p):
    cfg = gmg_box(dim, (4,) * dim, p, Pe=50.0)
    A, _ = _conc_block(cfg)
    P = mg.prolongation(cfg.n, p).toarray()
    Ad = A.toarray()
    Ac = P.T @ Ad @ P
    C = np.eye(len(Ad)) - P @ np.linalg.solve(Ac, P.T @ Ad)
    g = mg.GMG(A, cfg.n, p, max_elems=int(np.prod(cfg.n)) // 2 ** dim)
    assert g.levels == 2
    assert np.abs(g.A[1].toarray() - Ac).max() <= 1e-12 * np.abs(Ac).max()
    assert np.abs(C @ C - C).max() <= 1e-9 * np.abs(C).max()
    assert np.abs(P.T @ Ad @ C).max() <= 1e-9 * np.abs(Ad).max()


@pytest.mark.parametrize("dim,n,p", [(2, (8, 8), 1), (3, (4, 4, 4), 1), (2, (4, 4), 2)])
def test_vcycle_transpose_is_adjoint(dim, n, p):
    cfg = gmg_box(dim, n, p, Pe=200.0)
    A, _ = _conc_block(cfg)
    g = mg.GMG(A, n, p)
    assert g.levels >= 2
    rng = np.random.default_rng(5)
    r, w = rng.uniform(-1, 1, A.shape[0]), rng.uniform(-1, 1, A.shape[0])
    a = g.vcycle(r) @ w
    b = r @ g.vcycle(w, transpose=True)
    assert abs(a - b) <= 1e-12 * abs(a)


def test_vcycle_contracts_independently_of_h():
    """Diffusion-dominated block (Pe = 1): the V-cycle as a stationary iteration
    reduces the error by a factor that stays bounded as the grid is refined."""
    rates = []
    for n in ((8, 8), (16, 16)):
        cfg = gmg_box(2, n, 1, Pe=1.0)
        A, _ = _conc_block(cfg)
        g = mg.GMG(A, n, 1)
        rng = np.random.default_rng(7)
        xs = rng.uniform(-1, 1, A.shape[0])
        b = A @ xs
        x = np.zeros_like(b)
        errs = [np.linalg.norm(xs)]
        for _ in range(6):
            x = x + g.vcycle(b - A @ x)
            errs.append(np.linalg.norm(xs - x))
        rates.append((errs[-1] / errs[2]) ** (1 / 4))
    assert rates[0] < 0.25 and rates[1] < 0.25, rates
    assert rates[1] < 1.5 * rates[0] + 0.02, rates
