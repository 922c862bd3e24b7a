"""Pins of the ItI oracle (Appendix B) against what the mathematics fixes:

* polynomial exactness: with incoming impedance data g = u_n + i eta u of a
  degree-5 polynomial (traces of degree <= p - 3 are interpolated exactly
  between Gauss and Chebyshev points) and f = L u, the method reproduces u
  to rounding for variable, complex-valued coefficients;
* the paper's ItI test problem (eq. ItI_problem: Laplace u + (1 + e^{-50|x|^2})
  u = f, u_n + i u = g, u = e^{20 i x} + e^{30 i y}) converges at a rate of at
  least p - 2 in h (Section 5.1);
* eq. (ItI_D_inv): D^{-1} assembled from W = I - D12 D21 inverts D;
* a source given at solve time (linear upward pass) equals the source folded
  into the build.
"""
import numpy as np
import pytest

import workloads as W
from oracle import hps as H
from oracle import iti as I


def _robin(tree, bpts, u_fn):
    """u_n + i eta u with the outward normal of the root side of each point."""
    u, d = u_fn(bpts)
    ux, uy = d
    x, y = bpts[:, 0], bpts[:, 1]
    un = np.where(np.isclose(y, tree.lo), -uy,
                  np.where(np.isclose(x, tree.hi), ux, np.where(np.isclose(y, tree.hi), uy, -ux)))
    return un, u


def _poly_case(p, L, eta, complex_coeffs):
    tree = H.Tree(2, L)
    disc = H.LeafDisc(2, p)
    pts = tree.leaf_points(disc)
    x, y = pts[..., 0], pts[..., 1]
    c = np.zeros((tree.n_leaves, 6, p * p), dtype=complex if complex_coeffs else float)
    c[:, 0] = -(1 + 0.2 * np.sin(x + 2 * y))
    c[:, 1] = 0.1 * np.cos(x * y)
    c[:, 2] = -(1 + 0.2 * np.cos(x - y))
    c[:, 3] = 0.3 * np.cos(3 * y)
    c[:, 4] = -0.2 * np.sin(2 * x)
    c[:, 5] = -9.0 * (1 + 0.3 * np.sin(3 * x))
    if complex_coeffs:
        c[:, 5] = c[:, 5] + 2j * np.cos(y)          # absorbing medium
    u, d = W.poly5(pts)
    f = sum(c[:, t, :] * d[t] for t in range(6))
    bpts = tree.root_boundary_points(disc)
    un, ub = _robin(tree, bpts, lambda q: (W.poly5(q)[0], (W.poly5(q)[1][3], W.poly5(q)[1][4])))
    return tree, c, f, un + 1j * eta * ub, u


@pytest.mark.parametrize("p,L,eta,cplx", [(8, 1, 3.0, False), (8, 2, 1.0, True), (10, 2, 5.0, False)])
def test_polynomial_exactness(p, L, eta, cplx):
    tree, c, f, g, u = _poly_case(p, L, eta, cplx)
    op = I.build(tree, p, eta, c)
    err = np.abs(I.solve(op, g, f) - u).max() / np.abs(u).max()
    assert err < 1e-11, err


def _paper_problem(L, p):
    tree = H.Tree(2, L)
    disc = H.LeafDisc(2, p)
    pts = tree.leaf_points(disc)
    x, y = pts[..., 0], pts[..., 1]
    c = np.zeros((tree.n_leaves, 6, p * p))
    c[:, 0] = 1.0
    c[:, 2] = 1.0
    c[:, 5] = 1.0 + np.exp(-50 * (x ** 2 + y ** 2))
    u = np.exp(20j * x) + np.exp(30j * y)
    f = -400 * np.exp(20j * x) - 900 * np.exp(30j * y) + c[:, 5] * u
    bpts = tree.root_boundary_points(disc)

    def ufn(q):
        e1, e2 = np.exp(20j * q[:, 0]), np.exp(30j * q[:, 1])
        return e1 + e2, (20j * e1, 30j * e2)
    un, ub = _robin(tree, bpts, ufn)
    return tree, disc, c, f, un + 1j * ub, u


def test_paper_problem_converges():
    p = 8
    errs = []
    for L in (3, 4):
        tree, disc, c, f, g, u = _paper_problem(L, p)
        us = I.solve(I.build(tree, p, 1.0, c), g, f)
        ii = disc.Ii
        errs.append(np.abs(us[:, ii] - u[:, ii]).max() / np.abs(u[:, ii]).max())
    rate = np.log2(errs[0] / errs[1])
    assert errs[1] < 5e-3 and rate >= p - 2 - 0.5, (errs, rate)


def test_d_inverse_by_w_schur():
    tree, c, f, g, u = _poly_case(8, 1, 2.0, True)
    ops = I.ItiLeafOps(H.LeafDisc(2, 8), tree.leaf_r, 2.0)
    leaves = [I.leaf_solve(ops, c[i], f[i]) for i in range(4)]
    n = 6
    A, B, C, D, h_ext, h_int = I.merge_blocks([lf.T for lf in leaves], [lf.h for lf in leaves], n)
    Dinv = I.d_inverse(D, n)
    assert np.abs(Dinv @ D - np.eye(8 * n)).max() < 1e-12
    # D has the identity diagonal blocks that eq. (ItI_D_inv) relies on
    assert np.array_equal(D[:4 * n, :4 * n], np.eye(4 * n)) and np.array_equal(D[4 * n:, 4 * n:], np.eye(4 * n))


def test_source_split_equals_folded_source():
    tree, c, f, g, u = _poly_case(8, 2, 1.5, False)
    a = I.solve(I.build(tree, 8, 1.5, c), g, f)
    b = I.solve(I.build(tree, 8, 1.5, c, f=f), g)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()
