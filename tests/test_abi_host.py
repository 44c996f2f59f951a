"""Host-side checks of the C ABI: the library loads, exports every function the
header declares, and rejects bad arguments before touching the GPU."""
import ctypes as C
import os
import re

import pytest

from paper_2112_09271_amd import dgnp

HDR = os.path.join(os.path.dirname(__file__), "..", "include", "dgnp.h")


def _declared():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dgnp_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert "dgnp_setup" in names and "dgnp_adjoint" in names
    L = dgnp.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(dgnp.EXPORTED)


def _mesh(dim=3, n=(2, 2, 2)):
    m = dgnp.dgnp_mesh()
    m.dim = dim
    for i in range(3):
        m.n[i] = n[i]
        m.hi[i] = 1.0
    return m


def _species(z=(1.0, -1.0), D=(1.0, 1.0)):
    zz = (C.c_double * len(z))(*z)
    dd = (C.c_double * len(D))(*D)
    return dgnp.dgnp_species(len(z), zz, dd), (zz, dd)


@pytest.mark.parametrize("case", ["order", "dim", "ions", "zero_charge", "bc_kind", "no_data", "phi_free",
                                  "electrode_no_params", "electrode_phi_dirichlet", "electrode_bad_ion",
                                  "electrode_nan", "half_allocator"])
def test_setup_rejects_bad_arguments(case):
    """Every one of these is refused on the host before any GPU call."""
    mesh = _mesh()
    mesh.phi_bc[0] = 1   # a potential-Dirichlet face fixes the potential
    order = 2
    sp, keep = _species()
    vel = dgnp.dgnp_velocity()
    opt = dgnp.dgnp_options()
    opt.c_ip = 10.0
    el = dgnp.dgnp_electrode()
    el.ion, el.alpha_a, el.alpha_c = 1, 1.0, 1.0
    if case == "phi_free":
        mesh.phi_bc[0] = 0   # all-Neumann potential: singular, reported instead of solved
    elif case == "electrode_no_params":
        mesh.c_bc[2] = dgnp.DGNP_C_ELECTRODE
    elif case == "electrode_phi_dirichlet":
        mesh.c_bc[0] = dgnp.DGNP_C_ELECTRODE
        opt.electrode = C.pointer(el)
    elif case == "electrode_bad_ion":
        mesh.c_bc[2] = dgnp.DGNP_C_ELECTRODE
        el.ion = 5
        opt.electrode = C.pointer(el)
    elif case == "electrode_nan":
        mesh.c_bc[2] = dgnp.DGNP_C_ELECTRODE
        el.j0[2] = float("nan")
        opt.electrode = C.pointer(el)
    elif case == "half_allocator":
        opt.alloc = dgnp.ALLOC_FN(lambda n, ctx: None)
    if case == "order":
        order = 7
    elif case == "dim":
        mesh.dim = 4
    elif case == "ions":
        sp, keep = _species((1.0,), (1.0,))
    elif case == "zero_charge":
        sp, keep = _species((1.0, 0.0), (1.0, 1.0))
    elif case == "bc_kind":
        mesh.c_bc[0] = 9
    elif case == "no_data":
        mesh.c_bc[0] = 1   # Dirichlet face but no nodal data given
    ctx = C.c_void_p()
    code = dgnp.lib().dgnp_setup(C.byref(mesh), order, C.byref(sp), C.byref(vel), C.byref(opt), None,
                                 C.byref(ctx))
    assert code != dgnp.DGNP_OK
    assert ctx.value is None
    assert len(dgnp.lib().dgnp_last_error()) > 0
    if case == "electrode_nan":
        assert code == dgnp.DGNP_E_NONFINITE
    elif case != "no_data":
        assert code == dgnp.DGNP_E_ARG, (code, dgnp.lib().dgnp_last_error())


def test_null_arguments():
    L = dgnp.lib()
    assert L.dgnp_residual(None, None, None, None) == dgnp.DGNP_E_ARG
    assert L.dgnp_jacobian_apply(None, None, None, 0, 0, None) == dgnp.DGNP_E_ARG
    assert L.dgnp_solve(None, None, None, None) == dgnp.DGNP_E_ARG
    L.dgnp_destroy(None)
