"""Adjoint gradients on the GPU: autograd interface, and the full 16^3 cube
(64 seeded inflow nodes of species 1 and Pe) against central differences of
GPU solves with relative steps."""
import time

import numpy as np
import pytest

from oracle import solve as osolve
from tests.gpu_cases import gpu_available, pair
from workload import adjoint_params, boundary_data

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def test_autograd_matches_adjoint_and_oracle():
    import torch

    from paper_2112_09271_amd.autograd import DGNPObjective
    cfg, od, gp = pair("adj2d")
    g = torch.tensor(boundary_data(cfg), dtype=torch.float64, requires_grad=True)
    Pe = torch.tensor(cfg.Pe, dtype=torch.float64, requires_grad=True)
    J = DGNPObjective.apply(g, Pe, gp, dict(rtol=1e-12))
    J.backward()
    x_ref, _ = osolve.newton(od, tol=1e-14)
    J_ref, dg_ref, dpe_ref, _ = osolve.adjoint(od, x_ref)
    assert abs(J.item() - J_ref) <= 1e-9 * abs(J_ref)
    assert np.linalg.norm(g.grad.numpy() - dg_ref) <= 1e-7 * np.linalg.norm(dg_ref)
    assert abs(Pe.grad.item() - dpe_ref) <= 1e-7 * abs(dpe_ref)


def test_autograd_backward_uses_forward_parameters():
    """Two forwards on one problem with different data and Pe, then backward on
    the first: the gradients are those of the first parameter set (backward puts
    them back), and a Pe gradient comes back with Pe's dtype."""
    import torch

    from paper_2112_09271_amd.autograd import DGNPObjective
    cfg, _, gp = pair("adj2d", with_oracle=False)
    d1 = boundary_data(cfg)
    d2 = d1 * 1.1 + 0.05
    kw = dict(rtol=1e-12)
    g_ref = torch.tensor(d1, dtype=torch.float64, requires_grad=True)
    p_ref = torch.tensor(cfg.Pe, dtype=torch.float64, requires_grad=True)
    DGNPObjective.apply(g_ref, p_ref, gp, kw).backward()
    g1 = torch.tensor(d1, dtype=torch.float64, requires_grad=True)
    p1 = torch.tensor(cfg.Pe, dtype=torch.float32, requires_grad=True)
    g2 = torch.tensor(d2, dtype=torch.float64, requires_grad=True)
    p2 = torch.tensor(cfg.Pe * 1.3, dtype=torch.float64, requires_grad=True)
    J1 = DGNPObjective.apply(g1, p1, gp, kw)
    J2 = DGNPObjective.apply(g2, p2, gp, kw)
    J1.backward()
    assert p1.grad.dtype == torch.float32
    assert np.linalg.norm(g1.grad.numpy() - g_ref.grad.numpy()) <= 1e-9 * np.linalg.norm(g_ref.grad.numpy())
    assert abs(float(p1.grad) - float(p_ref.grad)) <= 1e-6 * abs(float(p_ref.grad))
    J2.backward()
    assert abs(J2.item() - J1.item()) > 1e-6 * abs(J1.item())
    assert np.linalg.norm(g2.grad.numpy() - g_ref.grad.numpy()) > 1e-6 * np.linalg.norm(g_ref.grad.numpy())
    # a float Pe (not a tensor) gets no gradient
    g3 = torch.tensor(d1, dtype=torch.float64, requires_grad=True)
    DGNPObjective.apply(g3, float(cfg.Pe), gp, kw).backward()
    assert np.linalg.norm(g3.grad.numpy() - g_ref.grad.numpy()) <= 1e-9 * np.linalg.norm(g_ref.grad.numpy())


def test_cube_adjoint_matches_central_differences():
    from paper_2112_09271_amd.dgnp import DGNP_F32, DGNP_F64
    cfg, _, gp = pair("cfg4", with_oracle=False)
    data = boundary_data(cfg)
    params = adjoint_params(cfg)
    x, st = gp.solve(rtol=1e-13)
    assert st.status == 0
    J0, dbc, dpe, lam, ast = gp.adjoint(x, rtol=1e-12)
    J0m, dbcm, dpem, _, _ = gp.adjoint(x, rtol=1e-12, prec=DGNP_F32)
    g64 = dbc[0, params]
    assert np.linalg.norm(dbcm[0, params] - g64) <= 1e-8 * np.linalg.norm(g64)

    # every perturbed solve starts from the paper's initial guess, as the base
    # solve (a warm start from the base solution would keep part of that
    # solution's own error in one of the two solves of a pair, which the central
    # difference then divides by 2h), and goes to 1e-13: each solve leaves an
    # error of about its final residual in J, and the difference divides it by
    # 2h = 2e-6 (mixed precision: the same FP64 residual test, faster)
    def J_at(bc, Pe):
        gp.set_params(bc, Pe)
        xx, s = gp.solve(rtol=1e-13, prec=DGNP_F32)
        assert s.status == 0
        return gp.objective(xx)

    # all 64 parameters; they form one gradient vector whose error is measured
    # against the vector's largest entry (single-node sensitivities are small)
    picks = params
    scale = np.abs(g64).max()
    worst = 0.0
    t0 = time.perf_counter()
    for j in picks:
        h = 1e-6 * max(1.0, abs(data[0, j]))
        bp, bm = data.copy(), data.copy()
        bp[0, j] += h
        bm[0, j] -= h
        fd = (J_at(bp, cfg.Pe) - J_at(bm, cfg.Pe)) / (2 * h)
        print(f"node {j}: adjoint {dbc[0, j]:.8e} fd {fd:.8e} ({time.perf_counter() - t0:.1f} s)", flush=True)
        worst = max(worst, abs(fd - dbc[0, j]) / scale)
    h = 1e-6 * cfg.Pe
    fd_pe = (J_at(data, cfg.Pe + h) - J_at(data, cfg.Pe - h)) / (2 * h)
    gp.set_params(data, cfg.Pe)
    print(f"cube adjoint: worst data rel err {worst:.2e}, dJ/dPe {dpe:.6e} vs fd {fd_pe:.6e}, "
          f"adjoint fgmres {ast.lin_its_total}")
    assert worst <= 1e-5
    assert abs(fd_pe - dpe) <= 1e-5 * abs(fd_pe)
