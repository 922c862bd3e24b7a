"""Adjoint of the HPS solve and gradients of a misfit with respect to the
PDE coefficients.  Test infrastructure only: nothing in the product path
imports this module.

The solve is linear in its data: u = G_f f + G_g g, with f the source sampled
on the leaf grids and g the Dirichlet data at the root's Gauss points.  The
adjoint maps a weight w (shaped like u) to lam_src = G_f^T w (shaped like f)
and lam_bdry = G_g^T w (shaped like g).  The paper leaves custom derivative
rules for its solver to future work (Section 6); this module is the plain
mathematics that such a rule must reproduce.

* ``dense_adjoint``  the definition: transpose of the composite collocation
  system that the HPS method eliminates exactly (the system of
  ``oracle.dense``), solved with a sparse LU.
* ``hps_adjoint``    the transposed HPS passes on an oracle operator: every
  step of the upward source pass and of the downward pass (Section 3.2,
  eqs. for g~, h and g_int) applied transposed, in reverse order.
* ``coeff_grad``     dJ/dc_t for the coefficients c_t of L = sum_t c_t d_t:
  the collocation rows at interior nodes are the only rows that contain the
  coefficients, so with K u = b and lam = K^{-T} grad_u J,
  dJ/dc_t(x_m) = -lam(m) (d_t u)(x_m) at interior nodes m and 0 at the nodes
  that boundary bordering replaces.
* ``observation``    interpolation of u at scattered points: the solution on
  a leaf is its tensor Chebyshev interpolant (the leaf discretisation of
  Section 2), evaluated by the barycentric formula.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from . import dense
from .hps import INTERFACES, LeafDisc, Operator, Tree, _child_index_sets
from .spectral import interp_matrix


# --------------------------------------------------------------------------
# definition: transposed composite system
# --------------------------------------------------------------------------
def _root_panel_index(tree: Tree, disc: LeafDisc, layout):
    """Row offset in root-boundary order of every boundary panel (matched by
    the coordinates of its Gauss points)."""
    rb = tree.root_boundary_points(disc)
    key = {tuple(np.round(x, 12)): k for k, x in enumerate(rb)}
    out = {}
    for pkey in layout["bnd_rows"]:
        (i, f), = layout["owners"][pkey]
        pts = dense._panel_points(tree, disc, i, f)
        out[pkey] = np.array([key[tuple(np.round(x, 12))] for x in pts])
    return out


def dense_adjoint(tree: Tree, p: int, coeffs: np.ndarray, w: np.ndarray):
    """w [nrhs, n_leaves, p^d] -> (lam_src [nrhs, n_leaves, p^d],
    lam_bdry [nrhs, n_root_bdry]) by solving K^T y = [w; 0]."""
    K, layout = dense.assemble(tree, p, coeffs, sparse=True)
    disc = layout["disc"]
    n_u, npts, nf = layout["n_u"], layout["npts"], layout["nf"]
    lu = spla.splu(K.T.tocsc())
    ridx = _root_panel_index(tree, disc, layout)
    nb_root = sum(len(v) for v in ridx.values())
    w = w if w.ndim == 3 else w[None]
    lam_src = np.zeros_like(w)
    lam_bdry = np.zeros((w.shape[0], nb_root))
    rows_per_leaf = disc.n_i + disc.n_e
    for r in range(w.shape[0]):
        rhs = np.zeros(K.shape[0])
        rhs[:n_u] = w[r].ravel()
        y = lu.solve(rhs)
        for i in range(tree.n_leaves):
            lam_src[r, i, disc.Ii] = y[i * rows_per_leaf:i * rows_per_leaf + disc.n_i]
        for pkey, row in layout["bnd_rows"].items():
            lam_bdry[r, ridx[pkey]] = y[row:row + nf]
    return lam_src, lam_bdry


# --------------------------------------------------------------------------
# transposed HPS passes
# --------------------------------------------------------------------------
def hps_adjoint(op: Operator, w: np.ndarray):
    """One weight w [n_leaves, p^d] -> (lam_src [n_leaves, p^d], lam_bdry).

    Forward solve (oracle.hps.solve with a source): leaf v = L_ii^{-1} f_int,
    h = Q v; upward g~ = -D^{-1} h_int, h_parent = (h_ext + B g~)[perm];
    downward g_int = S g_ext + g~, children boundary data from (g_ext,
    g_int); leaf u = Y g + v.  Each step below is the transpose of one of
    these, taken in reverse order."""
    d = op.tree.d
    nd = 2 ** d
    disc = op.disc
    # leaf output u = Y g + v
    gbar = [lf.Y.T @ w[i] for i, lf in enumerate(op.leaves)]
    vbar = [w[i].copy() for i in range(op.tree.n_leaves)]
    # downward pass, transposed: leaves -> root
    gtbar = [None] * len(op.levels)
    for lev in range(len(op.levels) - 1, -1, -1):
        nodes = op.levels[lev]
        up, gts = [], []
        for j, node in enumerate(nodes):
            n = node.n
            ext, inter = _child_index_sets(d, n)
            kids = gbar[nd * j: nd * j + nd]
            g_ext_bar = np.concatenate([kids[c][ext[c]] for c in range(nd)])
            g_int_bar = np.zeros(len(INTERFACES[d]) * n)
            for c in range(nd):
                for i, ii in inter[c].items():
                    g_int_bar[i * n:(i + 1) * n] += kids[c][ii]
            g_ext_bar = g_ext_bar + node.S.T @ g_int_bar
            gts.append(g_int_bar)                  # g~ enters g_int additively
            up.append(g_ext_bar[node.perm])        # g_ext[perm] = g_parent
        gtbar[lev] = gts
        gbar = up
    lam_bdry = gbar[0]
    # upward source pass, transposed: root -> leaves (the root's h is unused)
    hbar = [np.zeros_like(lam_bdry)]
    for lev, nodes in enumerate(op.levels):
        down = []
        for j, node in enumerate(nodes):
            n = node.n
            ext, inter = _child_index_sets(d, n)
            h_seg_bar = np.empty_like(hbar[j])
            h_seg_bar[node.perm] = hbar[j]         # h_parent = h_seg[perm]
            gt_bar = gtbar[lev][j] + node.B.T @ h_seg_bar
            h_int_bar = -sla.lu_solve(node.D_lu, gt_bar, trans=1)
            off = np.cumsum([0] + [len(e) for e in ext])
            for c in range(nd):
                hc = np.empty(2 * d * n)
                hc[ext[c]] = h_seg_bar[off[c]:off[c + 1]]
                for i, ii in inter[c].items():
                    hc[ii] = h_int_bar[i * n:(i + 1) * n]
                down.append(hc)
        hbar = down
    lam_src = np.zeros((op.tree.n_leaves, op.p ** d))
    for i, lf in enumerate(op.leaves):
        vb = vbar[i] + op.Qr.T @ hbar[i]           # h = Q v
        lam_src[i, disc.Ii] = sla.lu_solve(lf.lu, vb[disc.Ii], trans=1)
    return lam_src, lam_bdry


# --------------------------------------------------------------------------
# coefficient gradient
# --------------------------------------------------------------------------
def coeff_grad(tree: Tree, p: int, u: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """u, lam [nrhs, n_leaves, p^d] -> dJ/dc [n_leaves, n_terms, p^d], summed
    over the right-hand sides: -lam * (d_t u) at interior nodes, 0 on the
    leaf boundary nodes."""
    disc = LeafDisc(tree.d, p)
    ops = disc.term_ops(tree.leaf_r)
    u = u if u.ndim == 3 else u[None]
    lam = lam if lam.ndim == 3 else lam[None]
    out = np.zeros((tree.n_leaves, len(ops), p ** tree.d))
    for r in range(u.shape[0]):
        for i in range(tree.n_leaves):
            for t, Dt in enumerate(ops):
                out[i, t] -= lam[r, i] * (Dt @ u[r, i])
    out[:, :, disc.Ie] = 0.0
    return out


# --------------------------------------------------------------------------
# observation operator
# --------------------------------------------------------------------------
def containing_leaf(tree: Tree, x: np.ndarray) -> int:
    """Index of the leaf that contains x; on a shared edge or face the lowest
    index among the leaves that contain it."""
    r2 = 2.0 * tree.leaf_r
    best = None
    for i in range(tree.n_leaves):
        c = tree.leaf_corner(i)
        if np.all(x >= c - 1e-14) and np.all(x <= c + r2 + 1e-14):
            best = i
            break
    if best is None:
        raise ValueError(f"point {x} is outside the domain")
    return best


def observation(tree: Tree, p: int, xs: np.ndarray):
    """(leaf index [m], weights [m, p^d]) with u(x_m) = weights[m] . u[leaf[m]]
    (tensor barycentric interpolation on the containing leaf)."""
    disc = LeafDisc(tree.d, p)
    leaf = np.empty(len(xs), dtype=int)
    W = np.empty((len(xs), p ** tree.d))
    for m, x in enumerate(xs):
        i = containing_leaf(tree, x)
        leaf[m] = i
        ref = (x - tree.leaf_corner(i)) / tree.leaf_r - 1.0
        rows = [interp_matrix(disc.x, np.array([ref[a]]))[0] for a in range(tree.d)]
        wt = rows[tree.d - 1]
        for a in range(tree.d - 2, -1, -1):
            wt = np.kron(wt, rows[a])           # first coordinate fastest
        W[m] = wt
    return leaf, W


def misfit(u: np.ndarray, leaf: np.ndarray, W: np.ndarray, u_obs: np.ndarray) -> float:
    """J = sum_m (u(x_m) - u_obs_m)^2."""
    r = np.einsum("mk,mk->m", W, u[leaf]) - u_obs
    return float(r @ r)


def misfit_weight(u: np.ndarray, leaf: np.ndarray, W: np.ndarray, u_obs: np.ndarray) -> np.ndarray:
    """grad_u J = 2 E^T (E u - u_obs), shaped like u."""
    r = np.einsum("mk,mk->m", W, u[leaf]) - u_obs
    w = np.zeros_like(u)
    np.add.at(w, leaf, 2.0 * r[:, None] * W)
    return w
