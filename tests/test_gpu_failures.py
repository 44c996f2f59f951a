"""Failure paths of the solver, forced from the host: non-finite inputs are
reported as DGNP_E_NONFINITE, an exhausted Newton budget as DGNP_E_NOCONV, and
a problem whose potential no face fixes is refused at setup; after each, the
same context (or a new one) solves normally.  No kernel is made to fault."""
import numpy as np
import pytest

from tests.gpu_cases import gpu_available, pair
from workload import boundary_data, get_config

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def test_nan_in_initial_guess_is_reported():
    import torch

    from paper_2112_09271_amd.dgnp import DGNP_E_NONFINITE, DGNP_F32, DgnpError
    cfg, _, gp = pair("cfg2t", with_oracle=False)
    x0 = torch.full((gp.N,), 1.0, dtype=torch.float64, device=gp.device)
    x0[: gp.Nf] = 0.0
    x0[gp.Nf + 5] = float("nan")   # one entry, not the all-NaN request for the paper's guess
    with pytest.raises(DgnpError) as ei:
        gp.solve(x0=x0, prec=DGNP_F32)
    assert ei.value.code == DGNP_E_NONFINITE
    x, st = gp.solve(prec=DGNP_F32)
    assert st.status == 0


def test_nan_in_boundary_data_is_reported():
    from paper_2112_09271_amd.dgnp import DGNP_E_NONFINITE, DgnpError, Problem
    cfg = get_config("cfg2t")
    data = boundary_data(cfg)
    bad = data.copy()
    bad[0, 3] = float("nan")
    with pytest.raises(DgnpError) as ei:
        Problem(cfg, bad)
    assert ei.value.code == DGNP_E_NONFINITE
    gp = Problem(cfg, data)
    with pytest.raises(DgnpError) as ei:
        gp.set_params(bad, cfg.Pe)
    assert ei.value.code == DGNP_E_NONFINITE
    with pytest.raises(DgnpError) as ei:
        gp.set_params(data, float("inf"))
    assert ei.value.code == DGNP_E_NONFINITE
    x, st = gp.solve()
    assert st.status == 0


def test_newton_budget_exhausted_is_reported():
    from paper_2112_09271_amd.dgnp import DGNP_E_NOCONV, DGNP_F64, DgnpError
    cfg, _, gp = pair("cfg3s", with_oracle=False)
    with pytest.raises(DgnpError) as ei:
        gp.solve(max_newton=1, rtol=1e-12, prec=DGNP_F64)
    assert ei.value.code == DGNP_E_NOCONV
    x, st = gp.solve(rtol=1e-10, prec=DGNP_F64)
    assert st.status == 0 and st.newton_its > 1


def test_potential_not_fixed_is_refused():
    from paper_2112_09271_amd.dgnp import DGNP_E_ARG, DgnpError, Problem
    cfg = get_config("cfg2t").with_(phi_bc=(0,) * 6)
    with pytest.raises(DgnpError) as ei:
        Problem(cfg, boundary_data(cfg))
    assert ei.value.code == DGNP_E_ARG
    assert "potential" in str(ei.value)
