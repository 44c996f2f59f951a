"""Seeded random arrays (no discretisation arithmetic here).

* boundary_data: nodal inflow / Dirichlet concentrations, i.i.d. U[0.5, 1.5],
  shape [m-1][n_bnode], species outermost, in the canonical boundary-node order.
* adjoint_params: the 64 boundary-node indices (species 1) whose data are the
  differentiated parameters of the adjoint study.
* random_state: an operator-test linearisation point, field-major [m][N_f]:
  phi ~ 0.05 U[-1,1], c_k ~ 1 + 0.2 U[-1,1] (keeps the conductivity positive).
* random_vector: U[-1, 1] of length N.
"""
from __future__ import annotations

import numpy as np

from .configs import ADJOINT_SEED, N_ADJOINT_PARAMS, Config, n_boundary_nodes


def boundary_data(cfg: Config, seed: int | None = None) -> np.ndarray:
    nb = n_boundary_nodes(cfg)
    rng = np.random.default_rng(cfg.seed if seed is None else seed)
    return rng.uniform(0.5, 1.5, size=(cfg.m - 1, nb))


def adjoint_params(cfg: Config) -> np.ndarray:
    nb = n_boundary_nodes(cfg)
    rng = np.random.default_rng(ADJOINT_SEED)
    return np.sort(rng.choice(nb, N_ADJOINT_PARAMS, replace=False))


def n_dof_field(cfg: Config) -> int:
    E = int(np.prod(cfg.n))
    return E * (cfg.p + 1) ** cfg.dim


def random_state(cfg: Config, seed: int = 7) -> np.ndarray:
    nf = n_dof_field(cfg)
    rng = np.random.default_rng(seed)
    x = np.empty((cfg.m, nf))
    x[0] = 0.05 * rng.uniform(-1.0, 1.0, nf)
    for k in range(1, cfg.m):
        x[k] = 1.0 + 0.2 * rng.uniform(-1.0, 1.0, nf)
    return x.reshape(-1)


def random_vector(cfg: Config, seed: int = 8) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, cfg.m * n_dof_field(cfg))
