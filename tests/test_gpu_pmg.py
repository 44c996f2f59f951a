"""GPU tests of p-multigrid for the potential block (paper Sec. 4.2): the
order-p level smoothed matrix-free, the potential block re-discretised at
p = 1 as the next level, then the trilinear and aggregation levels."""
import numpy as np
import pytest

from tests.gpu_cases import gpu_available, host, pair, rel_err
from workload import random_state, random_vector

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.mark.parametrize("name", ["cfg2t", "cfg3s", "cfg1"])
@pytest.mark.parametrize("mode", ["P", "PG"])
def test_pmg_preconditioner_symmetric_and_transposed(name, mode):
    """With symmetric smoothing and restriction = prolongation^T the potential
    V-cycle is symmetric, and <P r, w> = <r, P^T w> for the whole block
    preconditioner, double and float."""
    from paper_2112_09271_amd import dgnp
    from paper_2112_09271_amd.dgnp import DGNP_F32, DGNP_F64
    cfg, _, gp = pair(name, with_oracle=False, phi_mg=getattr(dgnp, "DGNP_PHIMG_" + mode))
    x = random_state(cfg)
    gp.set_state(x, prec=DGNP_F32)
    r = random_vector(cfg, 61)
    w = random_vector(cfg, 62)
    for prec, tol in ((DGNP_F64, 1e-12), (DGNP_F32, 2e-5)):
        Pr = host(gp.precond_apply(r, prec=prec))
        Ptw = host(gp.precond_apply(w, prec=prec, transpose=True))
        a, b = Pr @ w, r @ Ptw
        assert abs(a - b) <= tol * np.linalg.norm(Pr) * np.linalg.norm(w), (prec, a, b)
    r0 = r.copy()
    r0[gp.Nf:] = 0.0
    w0 = w.copy()
    w0[gp.Nf:] = 0.0
    a = host(gp.precond_apply(r0))[: gp.Nf] @ w0[: gp.Nf]
    b = host(gp.precond_apply(w0))[: gp.Nf] @ r0[: gp.Nf]
    assert abs(a - b) <= 1e-12 * abs(a)


@pytest.mark.parametrize("name", ["cfg2t", "cfg3s"])
@pytest.mark.parametrize("mode", ["P", "PG"])
def test_pmg_solve_matches_q1_hierarchy(name, mode):
    """Newton-FGMRES with p-multigrid reaches the same discrete solution as with
    the trilinear-start potential hierarchy (the preconditioner changes the
    path, not the root), in double and mixed precision."""
    from paper_2112_09271_amd import dgnp
    from paper_2112_09271_amd.dgnp import DGNP_F32, DGNP_F64, DGNP_PHIMG_Q1
    cfg, _, g0 = pair(name, with_oracle=False, phi_mg=DGNP_PHIMG_Q1)
    _, _, g1 = pair(name, with_oracle=False, phi_mg=getattr(dgnp, "DGNP_PHIMG_" + mode))
    x0, st0 = g0.solve(rtol=1e-10, prec=DGNP_F64)
    for prec in (DGNP_F64, DGNP_F32):
        x1, st1 = g1.solve(rtol=1e-10, prec=prec)
        print(f"{name} {mode} prec={prec}: fgmres {st1.lin_its_total} (Q1 start {st0.lin_its_total})")
        assert st1.status == 0 and st1.res_final <= 1e-10 * st1.res0
        assert rel_err(host(x1), host(x0)) <= 1e-7


def test_phi_mg_automatic_choice_and_errors():
    """The automatic choice is the trilinear start at p <= 2 and Galerkin
    p-multigrid at p = 3 (identical results to asking for them); p-multigrid at
    p = 1 and unknown choices are argument errors."""
    from paper_2112_09271_amd.dgnp import (DGNP_E_ARG, DGNP_F32, DGNP_PHIMG_AUTO, DGNP_PHIMG_P, DGNP_PHIMG_PG,
                                           DGNP_PHIMG_Q1, DgnpError)
    for name, explicit in (("cfg2t", DGNP_PHIMG_Q1), ("cfg3s", DGNP_PHIMG_PG)):
        cfg, _, ga = pair(name, with_oracle=False, phi_mg=DGNP_PHIMG_AUTO)
        _, _, ge = pair(name, with_oracle=False, phi_mg=explicit)
        xa, sa = ga.solve(prec=DGNP_F32)
        xe, se = ge.solve(prec=DGNP_F32)
        assert sa.lin_its_total == se.lin_its_total
        assert np.array_equal(host(xa), host(xe))
    for name, mode in (("cfg1", 7), ("cfg2t", -1)):
        with pytest.raises(DgnpError) as ei:
            pair(name, with_oracle=False, phi_mg=mode)
        assert ei.value.code == DGNP_E_ARG
    with pytest.raises(DgnpError) as ei:
        pair("cfg1", with_oracle=False, phi_mg=DGNP_PHIMG_P, p=1)
    assert ei.value.code == DGNP_E_ARG


@pytest.mark.parametrize("name", ["cfg2t", "cfg3s"])
def test_matrix_free_potential_block_matches_oracle(name):
    """The matrix-free potential block (SIPG with tabulated kappa, used by the
    p-multigrid smoother) equals the potential-potential block of the oracle's
    Jacobian and the assembled blocks: FP64 to 1e-12, FP32 to 2e-5."""
    from paper_2112_09271_amd.dgnp import (DGNP_F32, DGNP_F64, DGNP_PHIMG_PG, DGNP_PHIOP_ASSEMBLED,
                                           DGNP_PHIOP_MATFREE)
    cfg, od, gp = pair(name, with_oracle=True, phi_mg=DGNP_PHIMG_PG)
    x = random_state(cfg)
    Nf = gp.Nf
    v = random_vector(cfg, 71)[:Nf].copy()
    J = od.jacobian(x).tocsr()
    ref = J[:Nf, :Nf] @ v
    for prec, tol in ((DGNP_F64, 1e-12), (DGNP_F32, 2e-5)):
        gp.set_state(x, prec=prec)
        y_mf = host(gp.phi_apply(v, prec=prec, kind=DGNP_PHIOP_MATFREE))
        y_as = host(gp.phi_apply(v, prec=prec, kind=DGNP_PHIOP_ASSEMBLED))
        assert rel_err(y_mf, ref) <= tol, (prec, rel_err(y_mf, ref))
        assert rel_err(y_as, ref) <= tol, (prec, rel_err(y_as, ref))
