"""Pins of the oracle's analytic velocity fields against properties that the
flow definitions fix, not against the formula itself.

Vortex (cube problems): the flow is the rotated gradient of the stream function
psi = sin(pi x) sin(pi y) / pi, u = (d psi/dy, -d psi/dx); so it is
divergence-free, tangential on all six faces of the unit cube (no inflow or
outflow anywhere, which is why the cube's boundary tags go by geometry), and
has no z component.  Checked at the oracle's own volume and face Gauss points
with finite differences of psi, which a sign slip or swapped component fails.

Poiseuille (channel problems): zero on the walls y = y_lo, y_hi, parabolic, with
mean velocity 1 over the channel height (Pe is the mean speed).
"""
import numpy as np

from oracle.problem import Problem
from workload import boundary_data, get_config


def _psi(pts):
    return np.sin(np.pi * pts[..., 0]) * np.sin(np.pi * pts[..., 1]) / np.pi


def _fd(f, pts, axis, h=1e-6):
    e = np.zeros(pts.shape[-1])
    e[axis] = h
    return (f(pts + e) - f(pts - e)) / (2 * h)


def _vortex_problem():
    cfg = get_config("cfg2t")
    return Problem(cfg, boundary_data(cfg), Pe=1.0)


def test_vortex_is_rotated_stream_function_gradient():
    pr = _vortex_problem()
    pts = pr.mesh.vol_points().reshape(-1, 3)
    u = pr.uhat(pts)
    assert np.max(np.abs(u[:, 0] - _fd(_psi, pts, 1))) < 1e-8
    assert np.max(np.abs(u[:, 1] + _fd(_psi, pts, 0))) < 1e-8
    assert np.max(np.abs(u[:, 2])) == 0.0
    # orientation at a point where both components are non-trivial
    q = np.array([[0.25, 0.25, 0.5]])
    assert np.allclose(pr.uhat(q), [[0.5, -0.5, 0.0]], atol=1e-15)


def test_vortex_is_divergence_free():
    pr = _vortex_problem()
    pts = pr.mesh.vol_points().reshape(-1, 3)
    div = sum(_fd(lambda x, i=i: pr.uhat(x)[..., i], pts, i) for i in range(3))
    assert np.max(np.abs(div)) < 1e-7


def test_vortex_is_tangential_on_every_face():
    pr = _vortex_problem()
    msh = pr.mesh
    for t in range(6):
        a, s = divmod(t, 2)
        fp = msh.face_points(msh.bfaces[t], a, -1 if s == 0 else 1).reshape(-1, 3)
        un = pr.uhat(fp)[:, a]
        assert np.max(np.abs(un)) < 1e-15, t
        # the tangential part is not zero everywhere on the x and y faces
        if a < 2:
            assert np.max(np.abs(pr.uhat(fp)[:, 1 - a])) > 0.5


def test_poiseuille_profile():
    cfg = get_config("cfg3s")
    pr = Problem(cfg, boundary_data(cfg), Pe=1.0)
    H = cfg.hi[1] - cfg.lo[1]
    y = np.linspace(cfg.lo[1], cfg.hi[1], 11)
    pts = np.stack([np.full_like(y, 0.3), y, np.full_like(y, 0.1)], axis=-1)
    u = pr.uhat(pts)
    assert abs(u[0, 0]) < 1e-15 and abs(u[-1, 0]) < 1e-15
    assert np.all(u[1:-1, 0] > 0) and np.all(u[:, 1:] == 0.0)
    # mean over the height is 1 (5-point Gauss rule is exact for the parabola)
    xg, wg = np.polynomial.legendre.leggauss(5)
    yg = cfg.lo[1] + 0.5 * H * (xg + 1)
    pts = np.stack([np.zeros_like(yg), yg, np.zeros_like(yg)], axis=-1)
    assert abs(0.5 * np.sum(wg * pr.uhat(pts)[:, 0]) - 1.0) < 1e-14
    # maximum 3/2 at mid-height
    mid = np.array([[0.0, cfg.lo[1] + H / 2, 0.0]])
    assert abs(pr.uhat(mid)[0, 0] - 1.5) < 1e-15
