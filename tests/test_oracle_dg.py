"""Pins of the oracle's residual and Jacobian against what the mathematics fixes."""
import numpy as np
import pytest

from oracle import solve
from oracle.dg import DG
from oracle.problem import Problem
from tests.oracle_cases import adj2d, make, poly_problem
from workload import boundary_data, random_state, random_vector
from workload.configs import VEL_CONST


def _interp(dg):
    """Nodal interpolant of the manufactured solution."""
    pts = dg.msh.node_points()
    return np.concatenate([dg.P.exact(f, pts).reshape(-1) for f in range(dg.m)])


@pytest.mark.parametrize("dim,p", [(2, 1), (2, 2), (2, 3), (3, 2)])
def test_consistency_exact_solution_in_Vh(dim, p):
    """An exact solution that lies in V_h with exactly integrated data makes the
    residual vanish: every face term is consistent and every jump is zero."""
    dg = poly_problem(dim, p)
    x = _interp(dg)
    r = dg.residual(x)
    scale = np.abs(dg.residual(np.zeros_like(x))).max()
    assert np.abs(r).max() <= 1e-12 * scale
    # ... and Newton from the standard initial guess returns the interpolant
    xs, hist = solve.newton(dg, tol=1e-13)
    assert np.abs(xs - x).max() < 1e-10


@pytest.mark.parametrize("case", ["cfg1", "cfg2t", "cfg3s", "adj2d"])
def test_jacobian_matches_central_differences(case):
    """R is affine in c at fixed phi and piecewise affine in phi at fixed c, so a
    central difference reproduces J v up to rounding (no kink is crossed for
    these random states at steps this small)."""
    dg = DG(Problem(adj2d(), boundary_data(adj2d()))) if case == "adj2d" else make(case)
    cfg = dg.P.cfg
    x = random_state(cfg)
    v = random_vector(cfg)
    jv = dg.jac_apply(x, v)
    for eps in (1e-6, 1e-7):
        fd = (dg.residual(x + eps * v) - dg.residual(x - eps * v)) / (2 * eps)
        assert np.linalg.norm(fd - jv) <= 1e-8 * np.linalg.norm(jv)
    # concentration-only directions: R is exactly affine, any step works
    vc = v.copy()
    vc[: dg.msh.Nf] = 0.0
    fd = dg.residual(x + vc) - dg.residual(x)
    assert np.linalg.norm(fd - dg.jac_apply(x, vc)) <= 1e-12 * np.linalg.norm(fd)
    # assembled matrix equals the matrix-free apply
    J = dg.jacobian(x)
    assert np.linalg.norm(J @ v - jv) <= 1e-13 * np.linalg.norm(jv)


def test_dR_dPe_and_dR_dg_match_differences():
    cfg = adj2d()
    g = boundary_data(cfg)
    x = random_state(cfg)
    base = DG(Problem(cfg, g))
    h = 1e-3 * cfg.Pe
    fd = (DG(Problem(cfg, g, Pe=cfg.Pe + h)).residual(x)
          - DG(Problem(cfg, g, Pe=cfg.Pe - h)).residual(x)) / (2 * h)
    an = base.dR_dPe(x)
    assert np.linalg.norm(fd - an) <= 1e-9 * np.linalg.norm(an)
    rng = np.random.default_rng(3)
    dgv = rng.uniform(-1, 1, g.shape)
    fd = DG(Problem(cfg, g + dgv)).residual(x) - base.residual(x)
    an = base.lin_apply(x, None, dg=dgv)
    assert np.linalg.norm(fd - an) <= 1e-12 * np.linalg.norm(an)
    lam = random_vector(cfg)
    assert np.allclose(base.dR_dg_T(x, lam).reshape(-1), lam @ base.dR_dg(x), rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("case", ["cfg1", "cfg2t"])
def test_sipg_potential_block_is_symmetric(case):
    dg = make(case)
    x = random_state(dg.P.cfg)
    Nf = dg.msh.Nf
    A = dg.jacobian(x, fields=[(0, 0)])[:Nf, :Nf]
    assert abs(A - A.T).max() <= 1e-14 * abs(A).max()
    # positive definite on random vectors
    v = random_vector(dg.P.cfg)[:Nf]
    assert v @ (A @ v) > 0


def test_concentration_block_symmetric_without_transport():
    """With u = 0 and a constant potential the concentration blocks reduce to SIPG
    diffusion and are symmetric."""
    dg = make("cfg2t", vel_kind=VEL_CONST, vel_param=(0.0, 0.0, 0.0))
    x = random_state(dg.P.cfg)
    Nf = dg.msh.Nf
    x[:Nf] = 0.3
    J = dg.jacobian(x)
    for k in (1, 2):
        A = J[k * Nf:(k + 1) * Nf, k * Nf:(k + 1) * Nf]
        assert abs(A - A.T).max() <= 1e-14 * abs(A).max()


def test_electroneutrality_by_construction():
    dg = make("cfg2t")
    x = random_state(dg.P.cfg)
    cm = solve.recover_cm(dg, x)
    X = dg.fields(x)
    z = dg.P.z
    tot = sum(z[k - 1] * X[k] for k in range(1, dg.m)) + z[-1] * cm
    mag = sum(abs(z[k - 1] * X[k]) for k in range(1, dg.m)) + abs(z[-1] * cm)
    assert np.all(np.abs(tot) <= 4 * np.finfo(float).eps * mag)


def test_global_species_balance_channel():
    """At the converged channel solution the species-1 outflow through x = x_max
    equals the inflow (u.n) c_in through x = 0; walls and electrodes carry no
    species-1 flux.  The inflow is integrated here independently with a
    10-point Gauss rule of the nodal data's own Lagrange interpolant."""
    dg = make("cfg3s", n=(4, 2, 2), hi=(1.0, 0.5, 0.5), Pe=50.0)
    xs, hist = solve.newton(dg, tol=1e-13)
    assert hist[-1] <= 1e-11 * hist[0]
    out = dg.objective(xs)
    cfg, msh, P = dg.P.cfg, dg.msh, dg.P
    xg, wg = np.polynomial.legendre.leggauss(10)
    nodes = np.polynomial.legendre.Legendre.basis(cfg.p).deriv().roots()
    nodes = np.concatenate([[-1.0], np.sort(nodes), [1.0]])

    def lag(j, t):
        out = np.ones_like(t)
        for i, xi in enumerate(nodes):
            if i != j:
                out = out * (t - xi) / (nodes[j] - xi)
        return out

    inflow = 0.0
    nfn = (cfg.p + 1) ** 2
    g = P.bc_conc[0]
    hy, hz = msh.h[1], msh.h[2]
    H = cfg.hi[1] - cfg.lo[1]
    for fi, e in enumerate(msh.bfaces[0]):
        iy, iz = msh.eidx[e, 1], msh.eidx[e, 2]
        ys = cfg.lo[1] + (iy + (xg + 1) / 2) * hy
        ux = 6 * cfg.Pe * ys * (H - ys) / H ** 2
        for j in range(nfn):
            jb, jc = j % (cfg.p + 1), j // (cfg.p + 1)
            val = np.einsum("i,j->ij", wg * ux * lag(jb, xg), wg * lag(jc, xg)).sum() * hy * hz / 4
            inflow += -val * g[fi * nfn + j]
    assert abs(out + inflow) <= 1e-9 * abs(inflow)
