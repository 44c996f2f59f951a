"""The optional inputs of dgnp_options: caller-supplied volume sources and
boundary data at the Gauss points (a manufactured problem posed from arrays,
solved against the oracle's own manufactured-solution solve), and a device
allocator hook backed by PyTorch's caching allocator."""
import numpy as np
import pytest

from oracle import solve as osolve
from tests.gpu_cases import gpu_available, host, pair
from workload import random_state, random_vector
from workload.configs import C_DIRICHLET, C_INFLOW, MMS_NONE

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _caller_arrays(od):
    """Sources at the volume Gauss points and boundary data at the face Gauss
    points of every boundary face, in the layout of dgnp_options, taken from the
    oracle's manufactured problem."""
    P, msh = od.P, od.msh
    m, d = P.m, P.dim
    vp = msh.vol_points()
    src = np.stack([P.source(f, vp) for f in range(m)])               # [m][E][nqv]
    rows = [[] for _ in range(m)]
    for t in range(2 * d):
        a, s = divmod(t, 2)
        n_e = len(msh.bfaces[t])
        nqf = msh.face_points(msh.bfaces[t][:1], a, -1 if s == 0 else 1).shape[1]
        rows[0].append(P.phi_data(t) if P.is_phi_dirichlet(t) else np.zeros((n_e, nqf)))
        for k in range(1, m):
            has = P.c_bc[t] in (C_DIRICHLET, C_INFLOW)
            rows[k].append(P.c_data(k, t) if has else np.zeros((n_e, nqf)))
    face = np.stack([np.concatenate(r, axis=0) for r in rows])        # [m][n_bface][nqf]
    return src, face


@pytest.mark.parametrize("name,kw", [("cfg1", {}), ("e1", dict(n=(4, 4, 4), p=2))])
def test_manufactured_problem_from_caller_arrays(name, kw):
    from paper_2112_09271_amd.dgnp import DGNP_F32, DGNP_F64, Problem
    cfg, od, _ = pair(name, **kw)
    src, face = _caller_arrays(od)
    gp = Problem(cfg.with_(mms=MMS_NONE), None, src_vol=src, dir_face=face)
    x_ref, _ = osolve.newton(od, tol=1e-13)
    for prec in (DGNP_F64, DGNP_F32):
        x, st = gp.solve(rtol=1e-11, prec=prec)
        err = np.linalg.norm(host(x) - x_ref) / np.linalg.norm(x_ref)
        print(f"{name} caller arrays prec={prec}: newton {st.newton_its}, fgmres {st.lin_its_total}, rel err {err:.2e}")
        assert st.status == 0 and err <= 1e-8
    # the residual posed from arrays equals the built-in manufactured residual
    xr = random_state(cfg)
    assert np.max(np.abs(host(gp.residual(xr)) - od.residual(xr))) <= 1e-12 * np.max(np.abs(od.residual(xr)))
    gp.close()


def test_torch_allocator_hook():
    import torch

    from paper_2112_09271_amd.dgnp import DGNP_F32, Problem, TorchAllocator
    from workload import boundary_data
    cfg, _, ref = pair("cfg3s", with_oracle=False)
    alloc = TorchAllocator()
    before = torch.cuda.memory_allocated()
    gp = Problem(cfg, boundary_data(cfg), allocator=alloc)
    x1, st1 = gp.solve(rtol=1e-10, prec=DGNP_F32)
    x0, st0 = ref.solve(rtol=1e-10, prec=DGNP_F32)
    assert st1.status == 0 and st0.status == 0
    assert np.array_equal(host(x1), host(x0))  # same kernels, same order: bitwise equal
    v = random_vector(cfg)
    assert np.array_equal(host(gp.jacobian_apply(v)), host(ref.jacobian_apply(v)))
    print(f"allocator hook: {alloc.n_alloc} allocations, {alloc.bytes_live / 2**20:.1f} MiB live, "
          f"torch allocated {(torch.cuda.memory_allocated() - before) / 2**20:.1f} MiB")
    assert alloc.n_alloc > 10 and alloc.bytes_live > 0
    assert torch.cuda.memory_allocated() - before >= alloc.bytes_live
    gp.close()
    assert alloc.live == {} and alloc.n_free == alloc.n_alloc
    ref.close()
