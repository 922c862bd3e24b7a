"""Pins of the oracle's 1D spectral building blocks (no GPU)."""
import numpy as np
import pytest

from oracle.spectral import (bary_weights, cheb_lobatto, diff_matrix,
                             gauss_legendre, interp_matrix)


@pytest.mark.parametrize("p", [3, 4, 8, 12, 16])
def test_cheb_nodes_closed_form(p):
    x = cheb_lobatto(p)
    assert x[0] == -1.0 and x[-1] == 1.0
    assert np.all(np.diff(x) > 0)
    # symmetric about 0 and the extrema of T_{p-1}: T_{p-1}(x_j) = (-1)^{p-1-j}
    np.testing.assert_allclose(x, -x[::-1], atol=1e-15)
    T = np.cos((p - 1) * np.arccos(np.clip(x, -1, 1)))
    np.testing.assert_allclose(np.abs(T), 1.0, atol=1e-13)
    if p == 3:
        np.testing.assert_array_equal(x, [-1.0, 0.0, 1.0])


@pytest.mark.parametrize("q", [1, 2, 4, 6, 10, 14])
def test_gauss_legendre_vs_library(q):
    x, w = gauss_legendre(q)
    xl, wl = np.polynomial.legendre.leggauss(q)
    np.testing.assert_allclose(x, xl, atol=1e-14)
    np.testing.assert_allclose(w, wl, atol=1e-14)
    assert abs(w.sum() - 2.0) < 1e-14
    # exact for every monomial of degree <= 2q - 1
    for k in range(2 * q):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-13


@pytest.mark.parametrize("p", [4, 8, 12, 16])
def test_diff_matrix_exact_on_polynomials(p):
    x = cheb_lobatto(p)
    D = diff_matrix(x)
    np.testing.assert_allclose(D.sum(axis=1), 0.0, atol=1e-11 * p * p)
    for k in range(p):
        np.testing.assert_allclose(D @ x ** k, k * x ** max(k - 1, 0) * (k > 0),
                                   atol=1e-11 * p ** 2)


def test_diff_matrix_textbook_corner_entries():
    # Classical Chebyshev differentiation matrix: for descending nodes the
    # (0,0) entry is (2N^2+1)/6; for ascending nodes it changes sign.
    for p in (5, 9, 16):
        N = p - 1
        D = diff_matrix(cheb_lobatto(p))
        assert abs(D[0, 0] + (2 * N * N + 1) / 6.0) < 1e-10
        assert abs(D[-1, -1] - (2 * N * N + 1) / 6.0) < 1e-10


def test_bary_weights_chebyshev_ratio():
    # Chebyshev--Lobatto barycentric weights are proportional to
    # (-1)^j delta_j with delta = 1/2 at the ends.
    p = 10
    w = bary_weights(cheb_lobatto(p))
    ref = np.array([(-1.0) ** j * (0.5 if j in (0, p - 1) else 1.0) for j in range(p)])
    ratio = w / ref
    np.testing.assert_allclose(ratio / ratio[0], 1.0, rtol=1e-12)


@pytest.mark.parametrize("p", [6, 12, 16])
def test_interpolation_exact(p):
    q = p - 2
    x = cheb_lobatto(p)
    g, _ = gauss_legendre(q)
    G2C = interp_matrix(g, x)
    C2G = interp_matrix(x, g)
    for k in range(q):            # degree <= q-1 from q Gauss points
        np.testing.assert_allclose(G2C @ g ** k, x ** k, atol=1e-12)
    for k in range(p):            # degree <= p-1 from p Chebyshev points
        np.testing.assert_allclose(C2G @ x ** k, g ** k, atol=1e-12)
    np.testing.assert_allclose(G2C.sum(axis=1), 1.0, atol=1e-13)
