"""The allocation-free objective entry point (dgnp_objective_noalloc) against
dgnp_objective through the C ABI: two calls in a row on one GPU, the second on a
smaller problem (the shared static partial-sum array keeps the first call's
larger contents), and the size limit rejected on the host."""
import ctypes as C

import numpy as np
import pytest

from tests.gpu_cases import gpu_available, pair
from workload import random_state

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _noalloc(gp, x):
    import torch

    from paper_2112_09271_amd import dgnp as D
    J = torch.full((1,), float("nan"), dtype=torch.float64, device=gp.device)
    D.dgnp_objective_noalloc(gp.ctx, x.data_ptr(), 0, J.data_ptr(), D._stream())
    torch.cuda.synchronize()
    return float(J.item())


def test_objective_noalloc_matches_objective_twice():
    import torch
    vals = []
    for name in ("cfg2", "cfg3s", "cfg2t"):  # 4096, then 64 and 64 elements
        cfg, _, gp = pair(name, with_oracle=False)
        x = torch.as_tensor(random_state(cfg), device=gp.device)
        J_ref = gp.objective(x)
        J = _noalloc(gp, x)
        J2 = _noalloc(gp, x)
        print(f"{name}: objective {J_ref:.15e}, allocation-free {J:.15e}")
        assert abs(J - J_ref) <= 1e-13 * abs(J_ref) + 1e-300
        assert J2 == J
        vals.append(J)
        gp.close()
    assert vals[0] != vals[2]


def test_objective_noalloc_rejects_large_problems():
    from paper_2112_09271_amd.dgnp import DGNP_E_ARG, DgnpError
    import torch
    cfg, _, gp = pair("e1", with_oracle=False, n=(128, 64, 33), p=1)  # 270,336 elements > 2^18
    x = torch.zeros(gp.N, dtype=torch.float64, device=gp.device)
    with pytest.raises(DgnpError) as ei:
        _noalloc(gp, x)
    assert ei.value.code == DGNP_E_ARG
    gp.close()
