"""Pins of the adaptive 3D oracle (Section 4.2) against the mathematics (no GPU).

* a uniform tree run through the non-uniform code is the uniform oracle, to the bit;
* a polynomial solution of degree p - 3 per variable is reproduced exactly on
  trees with level jumps across interfaces (the leaf discretization and both
  panel operators are exact there, so a wrong block, sign, orientation or
  quadrant in the projections breaks it);
* the panel operators reproduce polynomials and compose to the identity;
* the refinement criterion leaves polynomials of degree p - 1 unrefined, the
  refined tree meets the criterion on every leaf below the level cap, the
  level restriction holds after balancing, and balancing only adds splits;
* the root D sizes of uniform trees equal the table of Section 4.2.
"""
import os

import numpy as np
import pytest

import workloads as W
from oracle import adaptive as A
from oracle import hps
from test_oracle_hps import _var_coeffs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _poly(coef):
    def u_fun(x):
        out = np.zeros(x.shape[:-1])
        for idx in np.ndindex(*coef.shape):
            out += coef[idx] * np.prod([x[..., a] ** idx[a] for a in range(3)], axis=0)
        return out

    def deriv(x, orders):
        out = np.zeros(x.shape[:-1])
        for idx in np.ndindex(*coef.shape):
            term = coef[idx]
            for a in range(3):
                k, o = idx[a], orders[a]
                if k < o:
                    term = 0.0 * term
                    break
                fac = np.prod(np.arange(k - o + 1, k + 1)) if o else 1.0
                term = term * fac * x[..., a] ** (k - o)
            out = out + term
        return out

    return u_fun, deriv


def _apply_L(c, pts, deriv):
    ax = {"x": 0, "y": 1, "z": 2}
    f = np.zeros(pts.shape[:-1])
    for t, name in enumerate(W.TERMS_3D):
        orders = [0, 0, 0]
        if name != "0":
            for ch in name:
                orders[ax[ch]] += 1
        f += c[:, t, :] * deriv(pts, orders)
    return f


def _jump_tree(lo=-1.0, hi=1.0):
    """Depth 1 with octants 0 and 6 refined once more and one grandchild of
    octant 0 refined again: level jumps across interior interfaces at two
    merge levels, balanced."""
    leaves = set(A.AdaptiveTree.uniform(1, lo, hi).leaves)
    for k in [(1, 0, 0, 0), (1, 1, 1, 1)]:
        leaves.remove(k)
        leaves.update(A.children(k))
    k = (2, 1, 1, 1)
    leaves.remove(k)
    leaves.update(A.children(k))
    leaves = A.balance(leaves, lo, hi)
    return A.AdaptiveTree(leaves, lo, hi)


def test_uniform_tree_equals_uniform_oracle():
    p, depth = 6, 2
    t = A.AdaptiveTree.uniform(depth, -1.0, 1.0)
    tree = hps.Tree(3, depth)
    disc = hps.LeafDisc(3, p)
    pts = tree.leaf_points(disc)
    assert np.array_equal(pts, t.leaf_points(disc))
    c = _var_coeffs(pts)
    f = np.random.default_rng(1).normal(size=(tree.n_leaves, p ** 3))
    bp = tree.root_boundary_points(disc)
    g = np.sin(bp[:, 0]) + bp[:, 1] * bp[:, 2]
    u = hps.solve(hps.build(tree, p, c), g, f)
    aop = A.build(t, p, c)
    assert np.abs(A.root_boundary_points(aop) - bp).max() < 1e-15
    assert np.array_equal(A.solve(aop, g, f), u)


@pytest.mark.parametrize("p", [6, 7])
def test_polynomial_solution_exact_across_level_jumps(p):
    t = _jump_tree()
    assert A.is_balanced(t) and len({k[0] for k in t.leaves}) == 3
    deg = p - 3
    coef = np.random.default_rng(11).normal(size=(deg + 1,) * 3)
    u_fun, deriv = _poly(coef)
    disc = hps.LeafDisc(3, p)
    pts = t.leaf_points(disc)
    c = _var_coeffs(pts)
    f = _apply_L(c, pts, deriv)
    op = A.build(t, p, c)
    u = A.solve(op, u_fun(A.root_boundary_points(op)), f)
    ue = u_fun(pts)
    assert np.abs(u - ue).max() < 1e-10 * np.abs(ue).max()
    # the same with the source folded into the build
    op2 = A.build(t, p, c, f)
    u2 = A.solve(op2, u_fun(A.root_boundary_points(op2)))
    assert np.abs(u2 - ue).max() < 1e-10 * np.abs(ue).max()


def test_panel_operators_reproduce_polynomials():
    q = 5
    pan = A.Panels(q)
    g = pan.g
    G1, G2 = np.tile(g, q), np.repeat(g, q)
    rng = np.random.default_rng(3)
    cf = rng.normal(size=(q, q))

    def poly(a, b):
        return sum(cf[i, j] * a ** i * b ** j for i in range(q) for j in range(q))

    coarse = poly(G1, G2)
    fine = []
    for (s1, s2) in A.QUADRANTS:
        fine.append(poly((G1 + (2 * s1 - 1)) / 2.0, (G2 + (2 * s2 - 1)) / 2.0))
        assert np.allclose(pan.up[A.QUADRANTS.index((s1, s2))] @ coarse, fine[-1], atol=1e-12)
    assert np.allclose(pan.down @ np.concatenate(fine), coarse, atol=1e-12)
    assert np.allclose(pan.down @ np.vstack(pan.up), np.eye(q * q), atol=1e-12)


def test_seam_points_read_the_lower_quadrant():
    # odd q: the middle Gauss node sits on the seam between quadrants; its
    # four-to-one row uses the lower quadrant's panel (the reading stated in
    # the module docstring), whatever sign rounding gives the node
    q = 5
    pan = A.Panels(q)
    q2 = q * q
    mid = q // 2
    row = pan.down[mid + q * mid]
    assert np.count_nonzero(row[:q2]) > 0 and np.count_nonzero(row[q2:]) == 0
    row = pan.down[(q - 1) + q * mid]   # upper in t1, seam in t2 -> quadrant (1, 0)
    j = A.QUADRANTS.index((1, 0))
    assert np.count_nonzero(row[j * q2:(j + 1) * q2]) == np.count_nonzero(row) > 0


def test_refinement_leaves_polynomials_unrefined():
    p = 6
    f = lambda x: 1.0 + x[:, 0] ** 5 - 2.0 * x[:, 1] ** 3 * x[:, 2] ** 2 + x[:, 0] * x[:, 1] * x[:, 2]
    assert A.refine_one(f, p, 1e-12, 4) == {(0, 0, 0, 0)}


def _front(x, c=(0.52, 0.49, 0.51)):
    r = np.sqrt(((x - np.array(c)) ** 2).sum(axis=1))
    return np.arctan(10.0 * r - 0.7)


def test_refined_tree_meets_criterion_and_restriction():
    p, eps, cap = 6, 1e-3, 4
    leaves = A.refine_one(_front, p, eps, cap)
    t = A.AdaptiveTree(leaves)
    disc = hps.LeafDisc(3, p)
    L8 = A.child_interp(p)
    fnorm = max(np.abs(_front(t.points(disc, k))).max() for k in t.leaves)
    for k in t.leaves:
        if k[0] >= cap:
            continue
        x1 = np.concatenate([t.points(disc, ch) for ch in A.children(k)])
        assert np.abs(_front(x1) - L8 @ _front(t.points(disc, k))).max() < eps * fnorm
    assert len({k[0] for k in t.leaves}) >= 2
    bal = A.AdaptiveTree(A.balance(leaves))
    assert A.is_balanced(bal)
    # balancing only splits: every original leaf is a node of the balanced tree
    for k in leaves:
        assert k in bal.leafset or k in bal.internal
    # the union with a tree refined elsewhere refines both regions
    other = A.refine_one(lambda x: np.exp(-40.0 * ((x - 0.9) ** 2).sum(axis=1)), p, eps, 3)
    u = A.union([leaves, other])
    tu = A.AdaptiveTree(u)
    for k in list(leaves) + list(other):
        assert k in tu.leafset or k in tu.internal


def test_child_interpolation_matches_evaluation():
    p = 7
    disc = hps.LeafDisc(3, p)
    t = A.AdaptiveTree.uniform(0, 0.0, 1.0)
    f = lambda x: np.cos(x[:, 0] + 2 * x[:, 1]) * x[:, 2] ** 2
    root = (0, 0, 0, 0)
    x1 = np.concatenate([t.points(disc, ch) for ch in A.children(root)])
    # interpolating a degree-(p-1) polynomial is exact; a smooth function is close
    poly = lambda x: x[:, 0] ** 6 + x[:, 1] ** 3 * x[:, 2] ** 2 - x[:, 0] * x[:, 2]
    assert np.allclose(A.child_interp(p) @ poly(t.points(disc, root)), poly(x1), atol=1e-12)
    assert np.abs(A.child_interp(p) @ f(t.points(disc, root)) - f(x1)).max() < 1e-3


def test_root_D_sizes_uniform_match_paper_table():
    rows = np.loadtxt(os.path.join(GOLDEN, "merge_sizes_3d.txt"), dtype=int)
    for p, nleaves, size in rows:
        depth = {8: 1, 64: 2, 512: 3}[nleaves]
        if depth == 3 and p > 8:
            continue  # the size counts panels only; p = 8 at depth 3 already covers the walk
        assert A.root_D_size(A.AdaptiveTree.uniform(depth), p) == size


def test_adaptive_root_D_smaller_than_uniform():
    t = _jump_tree(0.0, 1.0)
    p = 8
    # one refined octant on each side of the root interfaces adds fine panels
    # only where both sides are fine
    assert A.root_D_size(t, p) < A.root_D_size(A.AdaptiveTree.uniform(t.max_level), p)
    assert A.root_D_size(t, p) >= A.root_D_size(A.AdaptiveTree.uniform(1), p)


def test_criterion_error_closed_form():
    # f = x^p on the unit cube: the degree-(p-1) interpolant through the p
    # Chebyshev-Lobatto nodes misses it by the nodal polynomial, so the
    # criterion's numerator is 2^-p max over the children's nodes y of
    # |prod_j (y - x_j)| (reference coordinates, x = (x_ref + 1) / 2)
    p = 6
    disc = hps.LeafDisc(3, p)
    t = A.AdaptiveTree.uniform(0, 0.0, 1.0)
    f = lambda x: x[:, 0] ** p
    root = (0, 0, 0, 0)
    x1 = np.concatenate([t.points(disc, ch) for ch in A.children(root)])
    err = np.abs(f(x1) - A.child_interp(p) @ f(t.points(disc, root))).max()
    xr = disc.x
    y = np.concatenate([(xr - 1.0) / 2.0, (xr + 1.0) / 2.0])
    nodal = np.array([np.prod(yy - xr) for yy in y])
    assert abs(err - 2.0 ** -p * np.abs(nodal).max()) < 1e-13
