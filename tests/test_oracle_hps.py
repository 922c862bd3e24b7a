"""Pins of the HPS oracle against the mathematics and the paper (no GPU).

Each test is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign or orientation, a transposed block, a mis-ordered segment) fails
at least one of them.
"""
import os

import numpy as np
import pytest

import workloads as W
from oracle import dense, hps

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _var_coeffs(pts, zeroth=True, mixed=True):
    """Smooth variable coefficients with every term switched on (2D/3D)."""
    d = pts.shape[-1]
    c = W.coeffs_poisson(pts)
    x = pts[..., 0]
    y = pts[..., 1]
    c[:, 0, :] = -(1.2 + 0.3 * np.sin(x + 2 * y))
    if d == 2:
        if mixed:
            c[:, 1, :] = 0.15 * np.cos(x * y)
        c[:, 3, :] = 0.4 * np.cos(3 * y)
        c[:, 4, :] = -0.3 * np.sin(2 * x)
    else:
        c[:, 6, :] = 0.4 * np.cos(3 * y)
        c[:, 8, :] = 0.2 * x
        if mixed:
            c[:, 3, :] = 0.1 * np.cos(x)
    if zeroth:
        c[:, -1, :] = -2.0 * (1.0 + 0.5 * np.sin(3 * x) * np.cos(y))
    return c


# ---------------------------------------------------------------------------
# P4: DtN invariants
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("d,p,L", [(2, 8, 0), (2, 10, 2), (3, 6, 0), (3, 5, 1)])
def test_T_annihilates_constants_without_zeroth_order_term(d, p, L):
    tree = hps.Tree(d, max(L, 1))
    disc = hps.LeafDisc(d, p)
    pts = tree.leaf_points(disc)
    c = _var_coeffs(pts, zeroth=False)
    op = hps.build(tree, p, c, root_T=True)
    ones = np.ones(disc.n_b)
    for lf in op.leaves:
        assert np.abs(lf.T @ ones).max() < 1e-9 * np.abs(lf.T).max()
    nb = op.root_T.shape[0]
    assert np.abs(op.root_T @ np.ones(nb)).max() < 1e-9 * np.abs(op.root_T).max()


@pytest.mark.parametrize("p", [8, 12])
def test_leaf_T_maps_harmonic_polynomial_to_normal_derivative(p):
    # Laplace leaf on [-1,1]^2: for u harmonic of degree <= p-3 per variable
    # (Re (x+iy)^k), T g = du/dn exactly at the Gauss points.
    tree = hps.Tree(2, 0)
    disc = hps.LeafDisc(2, p)
    pts = tree.leaf_points(disc)
    c = W.coeffs_poisson(pts)
    op_leaf = hps.leaf_solve(disc, disc.term_ops(1.0), disc.Q, c[0])
    bp = tree.leaf_boundary_points(disc, 0)
    normals = np.repeat(np.array([[0, -1], [1, 0], [0, 1], [-1, 0]], float),
                        disc.n_face, axis=0)
    for k in range(1, p - 2):
        z = bp[:, 0] + 1j * bp[:, 1]
        u = (z ** k).real
        du = k * z ** (k - 1)                 # u_x = Re, u_y = -Im
        grad = np.stack([du.real, -du.imag], axis=1)
        dn = np.sum(grad * normals, axis=1)
        np.testing.assert_allclose(op_leaf.T @ u, dn, atol=1e-9 * k ** 2 * 2 ** k)


def test_weighted_DtN_symmetry_improves_with_p():
    # Green's second identity for a self-adjoint operator: for smooth boundary
    # data g1, g2, <g1, T g2> = <T g1, g2> in L2(boundary).  With the Gauss
    # weights as the boundary quadrature the discrete asymmetry decays with
    # p (algebraically: the solution of a Dirichlet problem on a square has
    # corner singularities).  A sign or orientation slip leaves it O(1).
    asym = []
    for p in (6, 8, 10, 12):
        tree = hps.Tree(2, 0)
        disc = hps.LeafDisc(2, p)
        pts = tree.leaf_points(disc)
        c = W.coeffs_poisson(pts)
        c[0, -1, :] = -(1.0 + 0.5 * pts[0, :, 0] ** 2)      # -Laplace - k(x)
        lf = hps.leaf_solve(disc, disc.term_ops(1.0), disc.Q, c[0])
        bp = tree.leaf_boundary_points(disc, 0)
        g1 = np.cos(bp[:, 0] + 0.5 * bp[:, 1]) + bp[:, 1] ** 2
        g2 = np.exp(0.3 * bp[:, 0]) * np.sin(bp[:, 1] + 1.0)
        Wt = np.tile(disc.glw, 4)
        a, b = np.sum(Wt * g1 * (lf.T @ g2)), np.sum(Wt * (lf.T @ g1) * g2)
        asym.append(abs(a - b) / abs(a))
    assert all(x > y for x, y in zip(asym, asym[1:])), asym
    assert asym[-1] < asym[0] / 20 and asym[-1] < 1e-3, asym


# ---------------------------------------------------------------------------
# P5 / P6: against the dense composite collocation system
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("d_inverse", ["lu", "explicit"])
@pytest.mark.parametrize("d,p,L", [(2, 8, 2), (2, 7, 1), (3, 5, 1), (3, 4, 2)])
def test_full_solve_matches_dense_system(d, p, L, d_inverse):
    # both readings of "Invert D" (LU solves, explicit inverse) reach the
    # composite system's solution
    tree = hps.Tree(d, L)
    disc = hps.LeafDisc(d, p)
    pts = tree.leaf_points(disc)
    c = _var_coeffs(pts)
    f = np.sin(pts[..., 0] + 0.5) * np.cos(2 * pts[..., 1])
    gfun = lambda x: np.cos(x[..., 0]) + x[..., 1] ** 2 - 0.5 * x[..., -1]
    bp = tree.root_boundary_points(disc)
    op = hps.build(tree, p, c, f, d_inverse=d_inverse)
    u = hps.solve(op, gfun(bp))
    ud = dense.solve(tree, p, c, f, gfun)
    assert np.abs(u - ud).max() < 1e-11 * np.abs(ud).max()
    if d_inverse == "explicit":  # the solve-time source path uses the same inverse
        op2 = hps.build(tree, p, c, d_inverse=d_inverse)
        assert np.abs(hps.solve(op2, gfun(bp), f) - ud).max() < 1e-11 * np.abs(ud).max()


@pytest.mark.parametrize("d,p,L", [(2, 8, 1), (2, 6, 2), (3, 5, 1)])
def test_root_DtN_matches_dense_system(d, p, L):
    tree = hps.Tree(d, L)
    disc = hps.LeafDisc(d, p)
    pts = tree.leaf_points(disc)
    c = _var_coeffs(pts)
    gfun = lambda x: np.sin(x[..., 0] + 2 * x[..., 1]) + 0.3 * x[..., -1]
    bp = tree.root_boundary_points(disc)
    op = hps.build(tree, p, c, root_T=True)
    Tg = op.root_T @ gfun(bp)
    key = {tuple(np.round(x, 12)): k for k, x in enumerate(bp)}
    for P_, v in dense.root_dtn(tree, p, c, gfun):
        idx = [key[tuple(np.round(x, 12))] for x in P_]
        np.testing.assert_allclose(Tg[idx], v, atol=1e-10 * np.abs(Tg).max())


# ---------------------------------------------------------------------------
# P7: polynomial manufactured solutions are reproduced exactly
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("d,p,L", [(2, 8, 3), (2, 12, 2), (3, 6, 2)])
def test_polynomial_solution_exact(d, p, L):
    rng = np.random.default_rng(7)
    deg = p - 3
    coef = rng.normal(size=(deg + 1,) * d)

    def u_fun(x):
        out = np.zeros(x.shape[:-1])
        for idx in np.ndindex(*coef.shape):
            out += coef[idx] * np.prod([x[..., a] ** idx[a] for a in range(d)], axis=0)
        return out

    def deriv(x, orders):
        out = np.zeros(x.shape[:-1])
        for idx in np.ndindex(*coef.shape):
            term = coef[idx]
            for a in range(d):
                k, o = idx[a], orders[a]
                if k < o:
                    term = 0.0 * term
                    break
                fac = np.prod(np.arange(k - o + 1, k + 1)) if o else 1.0
                term = term * fac * x[..., a] ** (k - o)
            out = out + term
        return out

    tree = hps.Tree(d, L)
    disc = hps.LeafDisc(d, p)
    pts = tree.leaf_points(disc)
    c = _var_coeffs(pts)
    names = W.TERMS_2D if d == 2 else W.TERMS_3D
    ax = {"x": 0, "y": 1, "z": 2}
    f = np.zeros(pts.shape[:-1])
    for t, name in enumerate(names):
        orders = [0] * d
        if name != "0":
            for ch in name:
                orders[ax[ch]] += 1
        f += c[:, t, :] * deriv(pts, orders)
    bp = tree.root_boundary_points(disc)
    op = hps.build(tree, p, c)
    u = hps.solve(op, u_fun(bp), f)
    ue = u_fun(pts)
    assert np.abs(u - ue).max() < 1e-10 * np.abs(ue).max()


# ---------------------------------------------------------------------------
# P8: convergence on smooth manufactured solutions.  Spectral in p at fixed h.
# In h the printed construction (q = p - 2 Gauss points per side, bordering
# u(I_e) = P gamma, flux balance at the Gauss points) converges like h^(p-4)
# in the max norm, and the three tests below pin where the orders go:
#  * a leaf solved with the exact values at its Chebyshev boundary points is
#    off by O(h^p) (collocation alone);
#  * bordered from the exact Gauss values, P interpolates them with degree
#    q - 1 polynomials, so the leaf solution is off by O(h^(p-2)) (the
#    interpolation error h^q u^(q) times the nodal polynomial of the q Gauss
#    points);
#  * the normal derivative of that boundary error (it varies on the scale h)
#    leaves the flux-balance equations of the exact interface data with a
#    residual of O(h^(p-3)), whose smooth part is spread over 1/h interfaces
#    per unit length and acts like a volume source: the solution error is
#    O(h^(p-4)).
# ---------------------------------------------------------------------------
def _u_smooth(x):
    return np.sin(np.pi * x[..., 0]) * np.sin(np.pi * x[..., 1]) + np.exp(0.5 * x[..., 0]) * np.cos(0.7 * x[..., 1])


def _f_smooth(x):  # -Lap u
    return (2 * np.pi ** 2 * np.sin(np.pi * x[..., 0]) * np.sin(np.pi * x[..., 1])
            + 0.24 * np.exp(0.5 * x[..., 0]) * np.cos(0.7 * x[..., 1]))


def _consistency(p, L):
    """(global error, leaf error bordered from exact Gauss data, leaf error
    with exact Chebyshev boundary values, flux-balance residual of exact
    interface data), all relative to max |u|."""
    tree = hps.Tree(2, L)
    disc = hps.LeafDisc(2, p)
    pts = tree.leaf_points(disc)
    c = W.coeffs_poisson(pts)
    f = _f_smooth(pts)
    ue = _u_smooth(pts)
    sc = np.abs(ue).max()
    op = hps.build(tree, p, c)
    u = hps.solve(op, _u_smooth(tree.root_boundary_points(disc)), f)
    e_glob = np.abs(u - ue).max() / sc
    ops = disc.term_ops(tree.leaf_r)
    Qr = disc.Q / tree.leaf_r
    e_bord = e_exact = 0.0
    flux = {}
    q = disc.q
    for i in range(tree.n_leaves):
        lf = hps.leaf_solve(disc, ops, Qr, c[i], f[i])
        bp = tree.leaf_boundary_points(disc, i)
        ul = lf.Y @ _u_smooth(bp) + lf.v
        e_bord = max(e_bord, np.abs(ul - ue[i]).max() / sc)
        Lm = hps.leaf_operator(disc, ops, c[i])
        ux = ue[i].copy()
        ux[disc.Ii] = np.linalg.solve(Lm[np.ix_(disc.Ii, disc.Ii)],
                                      f[i][disc.Ii] - Lm[np.ix_(disc.Ii, disc.Ie)] @ ue[i][disc.Ie])
        e_exact = max(e_exact, np.abs(ux - ue[i]).max() / sc)
        qf = Qr @ ul
        for side in range(4):
            key = tuple(np.round(bp[side * q:(side + 1) * q].mean(0), 12))
            flux.setdefault(key, []).append(qf[side * q:(side + 1) * q])
    resid = max(np.abs(a + b).max() for a, b in (v for v in flux.values() if len(v) == 2))
    return np.array([e_glob, e_bord, e_exact, resid])


@pytest.fixture(scope="module")
def consistency_p8():
    p = 8
    errs = np.stack([_consistency(p, L) for L in (3, 4, 5)])
    return p, np.log2(errs[:-1] / errs[1:])          # rates between L = 3, 4, 5


def test_rate_global_error(consistency_p8):
    p, rates = consistency_p8
    assert rates[:, 0].min() > p - 4 - 0.25, rates[:, 0]


def test_rate_bordering_error(consistency_p8):
    p, rates = consistency_p8
    assert rates[:, 1].min() > p - 2 - 0.35, rates[:, 1]


def test_rate_exact_boundary_values(consistency_p8):
    p, rates = consistency_p8
    assert rates[0, 2] > p - 0.5, rates[:, 2]       # L = 5 reaches rounding


def test_rate_flux_residual(consistency_p8):
    p, rates = consistency_p8
    assert rates[:, 3].min() > p - 3 - 0.35 and rates[:, 3].max() < p - 3 + 0.35, rates[:, 3]


def _sinsin_error(p, L):
    tree = hps.Tree(2, L)
    disc = hps.LeafDisc(2, p)
    pts = tree.leaf_points(disc)
    c = W.coeffs_poisson(pts)
    bp = tree.root_boundary_points(disc)
    op = hps.build(tree, p, c)
    u = hps.solve(op, W.sinsin(bp), W.sinsin_minus_laplacian(pts))
    ue = W.sinsin(pts)
    return np.abs(u - ue).max() / np.abs(ue).max()


def test_spectral_convergence_in_p():
    errs = [_sinsin_error(p, 2) for p in (6, 8, 10, 12, 14)]
    assert all(b < a / 20 for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-10, errs


def test_convergence_variable_coefficient_problem():
    # eq. (DtN_problem), Section 5.1
    p = 10
    errs = []
    for L in (2, 3, 4):
        tree = hps.Tree(2, L)
        disc = hps.LeafDisc(2, p)
        pts = tree.leaf_points(disc)
        c = W.dtn_problem_coeffs(pts)
        f = W.dtn_problem_f(pts)
        bp = tree.root_boundary_points(disc)
        op = hps.build(tree, p, c)
        u = hps.solve(op, W.dtn_problem_u(bp), f)
        ue = W.dtn_problem_u(pts)
        errs.append(np.abs(u - ue).max() / np.abs(ue).max())
    rates = [np.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert min(rates) > p - 4 - 1.5 and errs[-1] < 1e-6, (errs, rates)


# ---------------------------------------------------------------------------
# P9: 3D merge sizes printed in the paper
# ---------------------------------------------------------------------------
def test_3d_root_D_sizes_match_paper_table():
    rows = [list(map(int, l.split())) for l in open(os.path.join(GOLDEN, "merge_sizes_3d.txt"))
            if l.strip() and not l.startswith("#")]
    for p, nleaves, Dsize in rows:
        depth = round(np.log(nleaves) / np.log(8))
        assert 8 ** depth == nleaves
        assert hps.merge_sizes(3, p, depth)[-1][1] == Dsize


@pytest.mark.parametrize("d,p,L", [(2, 6, 3), (3, 4, 2)])
def test_merge_sizes_match_built_blocks(d, p, L):
    tree = hps.Tree(d, L)
    disc = hps.LeafDisc(d, p)
    pts = tree.leaf_points(disc)
    op = hps.build(tree, p, _var_coeffs(pts), root_T=True)
    sizes = hps.merge_sizes(d, p, L)[::-1]          # root first
    for lev, nodes in enumerate(op.levels):
        nm, Dn, Tn = sizes[lev]
        assert len(nodes) == nm
        assert nodes[0].S.shape == (Dn, Tn)
    assert op.root_T.shape == (sizes[0][2],) * 2


# ---------------------------------------------------------------------------
# Merge block structure: literal App. A.2 blocks == general rule; 3D rule ==
# the pattern printed in App. C.2
# ---------------------------------------------------------------------------
def test_2d_literal_blocks_equal_general_rule():
    rng = np.random.default_rng(3)
    n = 5
    T = [rng.normal(size=(4 * n, 4 * n)) for _ in range(4)]
    h = [rng.normal(size=4 * n) for _ in range(4)]
    lit = hps.merge_blocks_2d(T, h, n)
    gen = hps.merge_blocks_general(2, T, h, n)
    for a, b in zip(lit, gen):
        np.testing.assert_array_equal(a, b)


def test_3d_block_pattern_matches_appendix_C2():
    names = "abcdefgh"
    want = set()
    for line in open(os.path.join(GOLDEN, "merge3d_pattern.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        m, r, c, *kids = line.split()
        want.add((m, int(r), int(c), "".join(sorted(kids))))
    got = set()
    touches = [dict() for _ in range(8)]
    for i, (c1, f1, c2, f2) in enumerate(hps.INTERFACES[3]):
        touches[c1][i + 9] = f1
        touches[c2][i + 9] = f2
    for c in range(8):
        for i in touches[c]:
            got.add(("B", c + 1, i, names[c]))
            got.add(("C", i, c + 1, names[c]))
    for i in range(9, 21):
        for j in range(9, 21):
            kids = [names[c] for c in range(8) if i in touches[c] and j in touches[c]]
            if kids:
                got.add(("D", i, j, "".join(sorted(kids))))
    assert got == want
    # and the interfaces are geometrically shared faces (opposite normals)
    for c1, f1, c2, f2 in hps.INTERFACES[3]:
        a1, s1, _ = hps.FACES[3][f1]
        a2, s2, _ = hps.FACES[3][f2]
        assert a1 == a2 and s1 != s2
        o1, o2 = hps.CHILD_OFFSETS[3][c1], hps.CHILD_OFFSETS[3][c2]
        diff = [o2[k] - o1[k] for k in range(3)]
        assert diff[a1] == (1 if s1 == 1 else -1) and sum(map(abs, diff)) == 1


# ---------------------------------------------------------------------------
# P10 / P12: source split, linearity, batching
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("d,p,L", [(2, 10, 2), (3, 5, 1)])
def test_source_split_equals_paper_form(d, p, L):
    tree = hps.Tree(d, L)
    disc = hps.LeafDisc(d, p)
    pts = tree.leaf_points(disc)
    c = _var_coeffs(pts)
    f = np.exp(pts[..., 0]) * np.sin(3 * pts[..., 1])
    g = np.cos(tree.root_boundary_points(disc)[:, 0])
    u_paper = hps.solve(hps.build(tree, p, c, f), g)
    u_split = hps.solve(hps.build(tree, p, c), g, f)
    assert np.abs(u_paper - u_split).max() < 1e-12 * np.abs(u_paper).max()


def test_linearity():
    tree = hps.Tree(2, 2)
    p = 8
    disc = hps.LeafDisc(2, p)
    pts = tree.leaf_points(disc)
    rng = np.random.default_rng(5)
    op = hps.build(tree, p, _var_coeffs(pts))
    nb = tree.root_boundary_points(disc).shape[0]
    g1, g2 = rng.normal(size=nb), rng.normal(size=nb)
    f1, f2 = rng.normal(size=pts.shape[:-1]), rng.normal(size=pts.shape[:-1])
    u12 = hps.solve(op, g1 + 2 * g2, f1 - f2)
    u_sum = hps.solve(op, g1, f1) + 2 * hps.solve(op, g2, 0 * f2) - hps.solve(op, 0 * g1, f2)
    assert np.abs(u12 - u_sum).max() < 1e-12 * np.abs(u12).max()


def test_point_layouts():
    tree = hps.Tree(2, 2)
    disc = hps.LeafDisc(2, 6)
    pts = tree.leaf_points(disc)
    # leaves 0..3 are the children a,b,c,d (SW, SE, NE, NW) of the SW quadrant
    centres = pts.mean(axis=1)
    np.testing.assert_allclose(centres[:4], [[-0.75, -0.75], [-0.25, -0.75],
                                             [-0.25, -0.25], [-0.75, -0.25]])
    # point order ix + p*iy, ascending
    assert np.all(np.diff(pts[0, :6, 0]) > 0) and np.all(pts[0, :6, 1] == pts[0, 0, 1])
    # root boundary order: S, E, N, W, ascending along each side
    bp = tree.root_boundary_points(disc)
    q = disc.q
    side = len(bp) // 4
    assert side == 4 * q
    S, E, N, Wd = bp[:side], bp[side:2 * side], bp[2 * side:3 * side], bp[3 * side:]
    assert np.all(S[:, 1] == -1) and np.all(np.diff(S[:, 0]) > 0)
    assert np.all(E[:, 0] == 1) and np.all(np.diff(E[:, 1]) > 0)
    assert np.all(N[:, 1] == 1) and np.all(np.diff(N[:, 0]) > 0)
    assert np.all(Wd[:, 0] == -1) and np.all(np.diff(Wd[:, 1]) > 0)


def test_merge_condition_estimate():
    # the oracle's per-merge condition record (LAPACK gecon on the LU
    # factors) against the exact 1-norm condition number of the same D
    import workloads as W
    tree = hps.Tree(2, 2)
    disc = hps.LeafDisc(2, 10)
    pts = tree.leaf_points(disc)
    c, _, _ = W.helmholtz_inputs(pts, tree.root_boundary_points(disc), 9.93, 1)
    op = hps.build(tree, 10, c)
    ops = disc.term_ops(tree.leaf_r)
    Qr = disc.Q / tree.leaf_r
    T, h = [], []
    for i in range(tree.n_leaves):
        lf = hps.leaf_solve(disc, ops, Qr, c[i], None)
        T.append(lf.T)
        h.append(lf.h)
    D = hps.merge_blocks_2d(T[0:4], h[0:4], disc.n_face)[3]
    exact = np.linalg.cond(D, 1)
    est = op.levels[1][0].cond1
    # gecon is a lower bound that is rarely off by more than a factor of 3
    assert exact / 3.0 <= est <= exact * (1 + 1e-8), (est, exact)
