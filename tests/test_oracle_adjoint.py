"""Pins of the adjoint / gradient oracle (no GPU).

The adjoint is fixed by the mathematics: for the linear solve map G,
<w, G a> = <G^T w, a> for every a and w; the coefficient gradient is the
derivative of the misfit, which central finite differences approximate to
O(h^2).  The pins use three independent routes: the transposed composite
system (definition), the transposed HPS passes, and the matrix of G built
column by column from the forward oracle solve (brute force).
"""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint as A
from oracle import dense, hps


def _coeffs(pts, seed=0, k=0.0):
    """Every term on, non-self-adjoint (first-order terms), seeded."""
    d = pts.shape[-1]
    g = np.random.default_rng(seed)
    a1, a2, a3 = g.uniform(0.5, 1.5, 3)
    x, y = pts[..., 0], pts[..., 1]
    c = W.coeffs_poisson(pts)
    c[:, 0, :] = -(1.0 + 0.2 * np.sin(a1 * x + 2 * y))
    if d == 2:
        c[:, 1, :] = 0.1 * np.cos(a2 * x * y)
        c[:, 2, :] = -(1.0 + 0.2 * np.cos(x - a3 * y))
        c[:, 3, :] = 0.3 * np.cos(3 * y)
        c[:, 4, :] = -0.2 * np.sin(2 * x)
    else:
        c[:, 3, :] = 0.1 * np.cos(x)
        c[:, 6, :] = 0.3 * np.cos(3 * y)
        c[:, 8, :] = 0.2 * x
    c[:, -1, :] = -(k * k) * (1.0 + 0.3 * np.sin(3 * x) * np.cos(y)) - 0.5
    return c


def _setup(d, p, L, seed=0, k=0.0):
    tree = hps.Tree(d, L)
    disc = hps.LeafDisc(d, p)
    pts = tree.leaf_points(disc)
    bpts = tree.root_boundary_points(disc)
    return tree, disc, pts, bpts, _coeffs(pts, seed, k)


def _gfun(bpts_all):
    wv = np.array([0.7, -1.3, 0.4])[: bpts_all.shape[-1]]
    return lambda x: np.cos(x @ wv) + 0.3 * x[..., 0]


@pytest.mark.parametrize("d,p,L", [(2, 6, 2), (2, 8, 1), (3, 5, 1)])
def test_dense_adjoint_dot_product(d, p, L):
    tree, disc, pts, bpts, c = _setup(d, p, L, seed=1)
    g = np.random.default_rng(7)
    f = g.normal(size=pts.shape[:-1])
    gfun = _gfun(bpts)
    u = dense.solve(tree, p, c, f, gfun)
    w = g.normal(size=u.shape)
    ls, lb = A.dense_adjoint(tree, p, c, w)
    lhs = np.sum(w * u)
    rhs_ = np.sum(ls[0] * f) + np.sum(lb[0] * gfun(bpts))
    assert abs(lhs - rhs_) < 1e-11 * max(abs(lhs), 1.0)
    assert np.all(ls[0][:, disc.Ie] == 0.0)


@pytest.mark.parametrize("d,p,L", [(2, 6, 2), (2, 8, 1), (2, 7, 3), (3, 5, 1), (3, 6, 1)])
def test_hps_adjoint_matches_definition(d, p, L):
    tree, disc, pts, bpts, c = _setup(d, p, L, seed=2, k=2.0)
    op = hps.build(tree, p, c)
    w = np.random.default_rng(3).normal(size=(2,) + pts.shape[:-1])
    ls_d, lb_d = A.dense_adjoint(tree, p, c, w)
    for r in range(2):
        ls, lb = A.hps_adjoint(op, w[r])
        assert np.abs(ls - ls_d[r]).max() < 1e-10 * np.abs(ls_d[r]).max()
        assert np.abs(lb - lb_d[r]).max() < 1e-10 * np.abs(lb_d[r]).max()


def test_hps_adjoint_brute_force_matrix():
    # G assembled column by column from the forward oracle solve
    d, p, L = 2, 5, 1
    tree, disc, pts, bpts, c = _setup(d, p, L, seed=4)
    op = hps.build(tree, p, c)
    nl, npts, nb = tree.n_leaves, p ** d, bpts.shape[0]
    cols_f = []
    for i in range(nl):
        for k in disc.Ii:
            f = np.zeros((nl, npts))
            f[i, k] = 1.0
            cols_f.append(hps.solve(op, np.zeros(nb), f).ravel())
    Gf = np.stack(cols_f, axis=1)
    Gg = np.stack([hps.solve(op, np.eye(nb)[j]).ravel() for j in range(nb)], axis=1)
    w = np.random.default_rng(5).normal(size=(nl, npts))
    ls, lb = A.hps_adjoint(op, w)
    ref_s = (Gf.T @ w.ravel()).reshape(nl, disc.n_i)
    assert np.abs(ls[:, disc.Ii] - ref_s).max() < 1e-11 * np.abs(ref_s).max()
    assert np.abs(lb - Gg.T @ w.ravel()).max() < 1e-11 * np.abs(lb).max()


def test_hps_adjoint_dot_product_helmholtz():
    d, p, L = 2, 10, 3
    tree = hps.Tree(d, L)
    disc = hps.LeafDisc(d, p)
    pts = tree.leaf_points(disc)
    bpts = tree.root_boundary_points(disc)
    c, bd, src = W.helmholtz_inputs(pts, bpts, 10.0, 1)
    op = hps.build(tree, p, c)
    u = hps.solve(op, bd[0], src[0])
    w = np.random.default_rng(6).normal(size=u.shape)
    ls, lb = A.hps_adjoint(op, w)
    lhs = np.sum(w * u)
    rhs_ = np.sum(ls * src[0]) + np.sum(lb * bd[0])
    assert abs(lhs - rhs_) < 1e-10 * np.sqrt(np.sum(w * w) * np.sum(u * u))


def _misfit_of(tree, p, c, bd, src, leaf, Wt, u_obs):
    op = hps.build(tree, p, c)
    u = hps.solve(op, bd, src)
    return A.misfit(u, leaf, Wt, u_obs), op, u


@pytest.mark.parametrize("d,p,L", [(2, 8, 2), (3, 5, 1)])
def test_coeff_grad_matches_finite_differences(d, p, L):
    tree, disc, pts, bpts, c = _setup(d, p, L, seed=8, k=1.5)
    g = np.random.default_rng(9)
    xs = g.uniform(-0.9, 0.9, size=(12, d))
    leaf, Wt = A.observation(tree, p, xs)
    bd = np.cos(bpts @ np.linspace(0.3, 1.1, d))
    src = np.exp(-np.sum(pts ** 2, axis=-1))
    u_obs = g.normal(size=len(xs)) * 0.1
    J0, op, u = _misfit_of(tree, p, c, bd, src, leaf, Wt, u_obs)
    w = A.misfit_weight(u, leaf, Wt, u_obs)
    ls, _ = A.hps_adjoint(op, w)
    grad = A.coeff_grad(tree, p, u[None], ls[None])
    nt = c.shape[1]
    checks = []
    for t in range(nt):                       # every term at an interior node
        checks.append((int(g.integers(tree.n_leaves)), t, int(disc.Ii[g.integers(disc.n_i)])))
    checks.append((0, nt - 1, int(disc.Ie[0])))   # a leaf boundary node: no dependence
    for (i, t, k) in checks:
        h = 1e-6 * max(1.0, abs(c[i, t, k]))
        cp, cm = c.copy(), c.copy()
        cp[i, t, k] += h
        cm[i, t, k] -= h
        Jp = _misfit_of(tree, p, cp, bd, src, leaf, Wt, u_obs)[0]
        Jm = _misfit_of(tree, p, cm, bd, src, leaf, Wt, u_obs)[0]
        fd = (Jp - Jm) / (2 * h)
        scale = np.abs(grad).max()
        assert abs(fd - grad[i, t, k]) < 1e-6 * scale, (i, t, k, fd, grad[i, t, k])
    assert np.all(grad[:, :, disc.Ie] == 0.0)


def test_misfit_weight_is_gradient_of_misfit():
    d, p, L = 2, 6, 2
    tree = hps.Tree(d, L)
    g = np.random.default_rng(10)
    xs = g.uniform(-0.9, 0.9, size=(9, d))
    leaf, Wt = A.observation(tree, p, xs)
    u = g.normal(size=(tree.n_leaves, p * p))
    v = g.normal(size=u.shape)
    u_obs = g.normal(size=9)
    # J is quadratic: J(u + e v) - J(u - e v) = 2 e <grad J, v> exactly
    e = 1e-3
    diff = A.misfit(u + e * v, leaf, Wt, u_obs) - A.misfit(u - e * v, leaf, Wt, u_obs)
    assert abs(diff - 2 * e * np.sum(A.misfit_weight(u, leaf, Wt, u_obs) * v)) < 1e-12


@pytest.mark.parametrize("d,p,L", [(2, 7, 2), (3, 5, 1)])
def test_observation_exact_for_polynomials(d, p, L):
    tree = hps.Tree(d, L)
    disc = hps.LeafDisc(d, p)
    pts = tree.leaf_points(disc)

    def poly(x):                      # degree p-1 in each variable
        out = np.ones(x.shape[:-1])
        for a in range(d):
            out = out * (x[..., a] ** (p - 1) - 0.5 * x[..., a] + 0.25 * a)
        return out

    u = poly(pts)
    xs = np.random.default_rng(11).uniform(-1, 1, size=(20, d))
    leaf, Wt = A.observation(tree, p, xs)
    vals = np.einsum("mk,mk->m", Wt, u[leaf])
    assert np.abs(vals - poly(xs)).max() < 1e-12 * np.abs(poly(xs)).max()


def test_observation_edge_point_goes_to_lowest_leaf():
    tree = hps.Tree(2, 2)
    p = 6
    for x in ([0.0, 0.0], [-0.5, 0.5], [0.5, -1.0], [1.0, 1.0]):   # leaf corners
        x = np.array(x)
        leaf, Wt = A.observation(tree, p, x[None])
        owners = [i for i in range(tree.n_leaves)
                  if np.all(x >= tree.leaf_corner(i) - 1e-14)
                  and np.all(x <= tree.leaf_corner(i) + 2 * tree.leaf_r + 1e-14)]
        assert leaf[0] == min(owners)
        # the point is a grid node of that leaf: the weights select it
        assert np.isclose(Wt[0].max(), 1.0) and np.isclose(np.abs(Wt[0]).sum(), 1.0)
