"""Shared helpers of the GPU parity tests: one config -> (oracle DG, GPU Problem)."""
import numpy as np
import pytest

from oracle.dg import DG
from oracle.problem import Problem as OProblem
from tests.oracle_cases import adj2d
from workload import boundary_data, get_config
from workload.configs import Config

torch = pytest.importorskip("torch")


def gpu_available():
    return torch.cuda.is_available()


def config(name, **kw):
    if isinstance(name, Config):
        cfg = name
    else:
        cfg = adj2d() if name == "adj2d" else get_config(name)
    return cfg.with_(**kw) if kw else cfg


def pair(name, with_oracle=True, phi_mg=0, **kw):
    from paper_2112_09271_amd.dgnp import Problem
    cfg = config(name, **kw)
    data = None if cfg.mms else boundary_data(cfg)
    print(f"[case] {cfg.name} n={cfg.n} p={cfg.p} m={cfg.m} phi_mg={phi_mg}", flush=True)
    gp = Problem(cfg, data, phi_mg=phi_mg)
    od = None
    if with_oracle:
        od = DG(OProblem(cfg) if cfg.mms else OProblem(cfg, data))
    return cfg, od, gp


def host(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()


def rel_err(a, b):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
