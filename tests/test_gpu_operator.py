"""Parity of the HIP DG operators with the CPU oracle (same seeded inputs)."""
import numpy as np
import pytest

from tests.gpu_cases import gpu_available, host, pair, rel_err
from workload import random_state, random_vector

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

SMALL = ["cfg1", "cfg2t", "cfg3s", "adj2d", "e1"]


@pytest.mark.parametrize("name", SMALL + ["cfg2"])
def test_connectivity_bit_exact(name):
    cfg, od, gp = pair(name)
    nbr, fe, fa, nbf = gp.connectivity()
    msh = od.msh
    assert np.array_equal(nbr, msh.nbr.astype(np.int32))
    assert np.array_equal(fe[:, 0], msh.face_minus) and np.array_equal(fe[:, 1], msh.face_plus)
    assert np.array_equal(fa, msh.face_axis)
    assert nbf == sum(len(v) for v in msh.bfaces.values())
    assert gp.n_bnode == od.P.n_bnode


@pytest.mark.parametrize("name", SMALL)
def test_residual_matches_oracle(name):
    cfg, od, gp = pair(name)
    for seed in (7, 17):
        x = random_state(cfg, seed)
        r_ref = od.residual(x)
        r = host(gp.residual(x))
        assert rel_err(r, r_ref) <= 1e-12


@pytest.mark.parametrize("name", SMALL)
def test_jacobian_and_transpose_match_oracle(name):
    cfg, od, gp = pair(name)
    x = random_state(cfg)
    v = random_vector(cfg)
    w = random_vector(cfg, 9)
    gp.set_state(x)
    jv = host(gp.jacobian_apply(v))
    assert rel_err(jv, od.jac_apply(x, v)) <= 1e-12
    J = od.jacobian(x)
    jtw = host(gp.jacobian_apply(w, transpose=True))
    assert rel_err(jtw, J.T @ w) <= 1e-12
    # dot-product test of the GPU pair
    assert abs(w @ jv - v @ jtw) <= 1e-13 * np.linalg.norm(w) * np.linalg.norm(jv)


@pytest.mark.parametrize("name", ["cfg2t", "cfg3s", "adj2d"])
def test_dR_dPe_matches_oracle(name):
    cfg, od, gp = pair(name)
    x = random_state(cfg)
    assert rel_err(host(gp.residual_dpe(x)), od.dR_dPe(x)) <= 1e-12


@pytest.mark.parametrize("name", ["cfg2t", "cfg3s"])
def test_float_apply_error(name):
    """The FP32 apply (FP32 state, FP32 arithmetic) stays within 2e-5 relative
    of the FP64 oracle at the seeded states."""
    from paper_2112_09271_amd.dgnp import DGNP_F32
    cfg, od, gp = pair(name)
    x = random_state(cfg)
    v = random_vector(cfg)
    gp.set_state(x, prec=DGNP_F32)
    ref = od.jac_apply(x, v)
    err32 = rel_err(host(gp.jacobian_apply(v, prec=DGNP_F32)), ref)
    print(f"fp32 apply max-rel error {err32:.3e}")
    assert err32 <= 2e-5


def test_full_size_cube_apply():
    """16^3, p = 2, three fields: full-size residual and Jacobian apply."""
    cfg, od, gp = pair("cfg2")
    x = random_state(cfg)
    v = random_vector(cfg)
    assert rel_err(host(gp.residual(x)), od.residual(x)) <= 1e-12
    gp.set_state(x)
    assert rel_err(host(gp.jacobian_apply(v)), od.jac_apply(x, v)) <= 1e-12


def test_bitwise_reproducible():
    cfg, od, gp = pair("cfg3s", with_oracle=False)
    x = random_state(cfg)
    v = random_vector(cfg)
    gp.set_state(x)
    a = host(gp.jacobian_apply(v))
    b = host(gp.jacobian_apply(v))
    assert np.array_equal(a, b)


@pytest.mark.parametrize("name", ["cfg2t", "cfg3s", "e1", "cfg1"])
def test_coupling_block_matches_oracle(name):
    """A_phi,c v_c (the coupling of Eq. P2): the potential rows of the oracle's
    J applied to v with its potential part zeroed, in FP64 (1e-12) and FP32."""
    from paper_2112_09271_amd.dgnp import DGNP_F32, DGNP_F64
    cfg, od, gp = pair(name)
    x = random_state(cfg)
    v = random_vector(cfg)
    vc = v.copy()
    vc[: gp.Nf] = 0.0
    ref = od.jac_apply(x, vc)[: gp.Nf]
    gp.set_state(x, prec=DGNP_F32)
    e64 = rel_err(host(gp.coupling_apply(v)), ref)
    e32 = rel_err(host(gp.coupling_apply(v, prec=DGNP_F32)), ref)
    print(f"{name}: coupling FP64 {e64:.2e}, FP32 {e32:.2e}")
    assert e64 <= 1e-12 and e32 <= 2e-5


@pytest.mark.parametrize("name", ["cfg2t", "cfg3s"])
def test_tabulated_apply_matches_general_kernel(name, monkeypatch):
    """The 3-D apply with tabulated linearisation data against the general
    operator kernel (which interpolates the state on every apply), both
    precisions, masked inputs included."""
    from paper_2112_09271_amd.dgnp import DGNP_F32, DGNP_F64
    cfg = pair(name, with_oracle=False)[0]
    x = random_state(cfg)
    v = random_vector(cfg)
    out = {}
    for general in (False, True):
        if general:
            monkeypatch.setenv("DGNP_JAC_GENERAL", "1")
        _, _, gp = pair(name, with_oracle=False)
        gp.set_state(x, prec=DGNP_F32)
        out[general] = [host(gp.jacobian_apply(v)), host(gp.jacobian_apply(v, prec=DGNP_F32)),
                        host(gp.coupling_apply(v)), host(gp.coupling_apply(v, prec=DGNP_F32))]
        gp.close()
    for i, (a, b) in enumerate(zip(out[False], out[True])):
        assert rel_err(a, b) <= (1e-12 if i % 2 == 0 else 1e-5), i
