"""Parity at the full sizes of the two channel workloads (64x16x8 and 128x32x16
hexes, p = 3, Poiseuille flow at Pe = 1e4, electrodes as fixed-potential faces;
1.57M and 12.6M DOFs), where the oracle's direct solver cannot run:

* the residual and the Jacobian apply against the oracle's vectorised ones,
  element by element (FP64 to 1e-12, the FP32 apply to 2e-5);
* the oracle's own residual at the GPU's converged FP64 and mixed-precision
  solutions (relative to the initial residual, which the first check pins);
* the FP64 and the mixed-precision solutions against each other.
"""
import numpy as np
import pytest

from tests.gpu_cases import gpu_available, host, pair, rel_err
from workload import random_state, random_vector

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


@pytest.mark.parametrize("name", ["cfg3", "cfg5"])
def test_channel_operators_full_size(name):
    from paper_2112_09271_amd.dgnp import DGNP_F32, DGNP_F64, DGNP_STATE_APPLY_ONLY
    cfg, od, gp = pair(name)
    x = random_state(cfg)
    v = random_vector(cfg)
    e_r = rel_err(host(gp.residual(x)), od.residual(x))
    jv_ref = od.jac_apply(x, v)
    gp.set_state(x, prec=DGNP_F64 | DGNP_STATE_APPLY_ONLY)
    e_j = rel_err(host(gp.jacobian_apply(v)), jv_ref)
    gp.set_state(x, prec=DGNP_F32 | DGNP_STATE_APPLY_ONLY)
    e_j32 = rel_err(host(gp.jacobian_apply(v, prec=DGNP_F32)), jv_ref)
    print(f"{name}: residual {e_r:.2e}, J apply FP64 {e_j:.2e}, FP32 {e_j32:.2e}")
    assert e_r <= 1e-12 and e_j <= 1e-12 and e_j32 <= 2e-5


@pytest.mark.parametrize("name,rtol", [("cfg3", 1e-10), ("cfg5", 1e-9)])
def test_channel_solutions_full_size(name, rtol):
    from paper_2112_09271_amd.dgnp import DGNP_F32, DGNP_F64
    cfg, od, gp = pair(name)
    sols = {}
    for prec in (DGNP_F32, DGNP_F64):
        x, st = gp.solve(rtol=rtol, prec=prec)
        print(f"{name} prec={prec}: newton {st.newton_its}, fgmres {st.lin_its_total}, refine "
              f"{st.refine_its_total}, |R| {st.res0:.3e}->{st.res_final:.3e}, t {st.t_total:.2f}s", flush=True)
        assert st.status == 0 and st.res_final <= rtol * st.res0
        xs = host(x)
        del x
        r = np.linalg.norm(od.residual(xs))
        print(f"  oracle |R(x_gpu)| / |R0| = {r / st.res0:.2e}", flush=True)
        assert r <= 2 * rtol * st.res0
        sols[prec] = xs
    d = _rel(sols[DGNP_F32], sols[DGNP_F64])
    print(f"{name}: FP64 vs mixed {d:.2e}")
    assert d <= 1e-8
