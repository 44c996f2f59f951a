"""Pin of the oracle's adjoint gradients against central differences of full solves."""
import numpy as np

from oracle import solve
from oracle.dg import DG
from oracle.problem import Problem
from tests.oracle_cases import adj2d
from workload import boundary_data


def _J(cfg, g, Pe):
    dg = DG(Problem(cfg, g, Pe=Pe))
    x, hist = solve.newton(dg, tol=1e-14)
    return dg.objective(x)


def test_adjoint_gradients_match_central_differences():
    cfg = adj2d()
    g = boundary_data(cfg)
    dg = DG(Problem(cfg, g))
    x, hist = solve.newton(dg, tol=1e-14)
    J0, dJdg, dJdPe, lam = solve.adjoint(dg, x)
    assert abs(J0 - dg.objective(x)) == 0.0
    assert J0 > 0  # species 1 (z = +1) leaves through x = 1 under the applied field
    rng = np.random.default_rng(11)
    picks = [(k, j) for k in range(cfg.m - 1) for j in rng.choice(g.shape[1], 2, replace=False)]
    for k, j in picks:
        h = 1e-6 * max(1.0, abs(g[k, j]))
        gp, gm = g.copy(), g.copy()
        gp[k, j] += h
        gm[k, j] -= h
        fd = (_J(cfg, gp, cfg.Pe) - _J(cfg, gm, cfg.Pe)) / (2 * h)
        assert abs(fd - dJdg[k, j]) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(dJdg).max())
    h = 1e-6 * max(1.0, cfg.Pe)
    fd = (_J(cfg, g, cfg.Pe + h) - _J(cfg, g, cfg.Pe - h)) / (2 * h)
    assert abs(fd - dJdPe) <= 1e-5 * abs(fd)
