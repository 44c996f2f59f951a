"""Pins of the oracle's reference rules: closed forms, exactness, Lagrange identities."""
import numpy as np
import pytest

from oracle.quadrature import gauss_legendre, gll_points, lagrange


def test_gll_closed_forms():
    assert np.allclose(gll_points(1), [-1.0, 1.0], atol=0)
    assert np.allclose(gll_points(2), [-1.0, 0.0, 1.0], atol=1e-15)
    assert np.allclose(gll_points(3), [-1.0, -1 / np.sqrt(5), 1 / np.sqrt(5), 1.0], atol=1e-15)
    # p = 4: 0, +-sqrt(3/7)
    assert np.allclose(gll_points(4), [-1, -np.sqrt(3 / 7), 0, np.sqrt(3 / 7), 1], atol=1e-14)


@pytest.mark.parametrize("nq", [2, 3, 4, 5, 6])
def test_gauss_exactness(nq):
    x, w = gauss_legendre(nq)
    for k in range(2 * nq):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * x ** k) - exact) < 1e-14
    # first degree that is not integrated exactly
    k = 2 * nq
    assert abs(np.sum(w * x ** k) - 2.0 / (k + 1)) > 1e-6


@pytest.mark.parametrize("p", [1, 2, 3])
def test_lagrange_identities(p):
    xn = gll_points(p)
    V, D = lagrange(xn, xn)
    assert np.allclose(V, np.eye(p + 1), atol=1e-15)
    pts = np.linspace(-1, 1, 13)
    V, D = lagrange(xn, pts)
    assert np.allclose(V.sum(1), 1.0, atol=1e-14)
    assert np.allclose(D.sum(1), 0.0, atol=1e-13)
    # interpolation and differentiation are exact on polynomials of degree <= p
    for k in range(p + 1):
        assert np.allclose(V @ xn ** k, pts ** k, atol=1e-14)
        dk = k * pts ** (k - 1) if k > 0 else 0 * pts
        assert np.allclose(D @ xn ** k, dk, atol=1e-13)
