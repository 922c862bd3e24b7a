"""The composite spectral collocation system that HPS solves, assembled and
solved densely (tiny trees only).  Test infrastructure only.

In exact arithmetic the HPS build and downward pass eliminate exactly this
linear system, block by block (Section 3: the local solves enforce the PDE on
interior Chebyshev nodes with boundary bordering; the merges enforce a single
boundary value on each shared panel and the balance of outward normal
derivatives across it, Appendix A.2 / C.2).  Assembling it directly, with no
Schur complements, gives an independent check of the whole oracle.

Unknowns: u on every Chebyshev node of every leaf, and gamma (the Gauss-point
boundary values) on every distinct leaf face ("panel").  Equations:

* E1  (L^(i) u_i)(m) = f_i(m) for interior nodes m of every leaf;
* E2  u_i(I_e) = P [gamma of leaf i's faces]  (boundary bordering);
* E3  (Q u_a) + (Q u_b) = 0 on every panel shared by leaves a and b
      (outward normal derivatives balance);
* gamma = g on panels that lie on the domain boundary.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sps

from .hps import FACES, LeafDisc, Tree, leaf_operator


def _panel_key(tree: Tree, i: int, f: int):
    cell = np.rint((tree.leaf_corner(i) - tree.lo) / (2 * tree.leaf_r)).astype(int)
    axis, side, tang = FACES[tree.d][f]
    return (axis, int(cell[axis] + side)) + tuple(int(cell[t]) for t in tang)


def assemble(tree: Tree, p: int, coeffs: np.ndarray, sparse: bool = False):
    """Returns (K, layout) with K the square system matrix (a dense array, or
    a scipy CSC matrix when ``sparse``; the entries are the same)."""
    d = tree.d
    disc = LeafDisc(d, p)
    ops = disc.term_ops(tree.leaf_r)
    Qr = disc.Q / tree.leaf_r
    npts = p ** d
    nf = disc.n_face
    panels = {}
    owners = {}
    for i in range(tree.n_leaves):
        for f in range(2 * d):
            key = _panel_key(tree, i, f)
            if key not in panels:
                panels[key] = len(panels)
                owners[key] = []
            owners[key].append((i, f))
    n_u = tree.n_leaves * npts
    n_unk = n_u + len(panels) * nf
    # every entry of K is written by exactly one of the blocks below
    blocks = []          # (row indices, column indices, dense block)

    def put(r0, nr, cols, blk):
        blocks.append((np.arange(r0, r0 + nr), np.asarray(cols), np.asarray(blk, dtype=float)))

    row = 0
    for i in range(tree.n_leaves):
        L = leaf_operator(disc, ops, coeffs[i])
        cu = np.arange(i * npts, (i + 1) * npts)
        # E1
        put(row, disc.n_i, cu, L[disc.Ii])
        row += disc.n_i
        # E2
        put(row, disc.n_e, i * npts + np.asarray(disc.Ie), np.eye(disc.n_e))
        for f in range(2 * d):
            pc = n_u + panels[_panel_key(tree, i, f)] * nf
            put(row, disc.n_e, np.arange(pc, pc + nf), -disc.P[:, f * nf:(f + 1) * nf])
        row += disc.n_e
    bnd_rows = {}
    for key, own in owners.items():
        pc = n_u + panels[key] * nf
        if len(own) == 2:              # E3
            for (i, f) in own:
                put(row, nf, np.arange(i * npts, (i + 1) * npts), Qr[f * nf:(f + 1) * nf])
        else:                          # gamma = g
            put(row, nf, np.arange(pc, pc + nf), np.eye(nf))
            bnd_rows[key] = row
        row += nf
    assert row == n_unk
    layout = dict(panels=panels, owners=owners, bnd_rows=bnd_rows, disc=disc,
                  n_u=n_u, nf=nf, npts=npts)
    if sparse:
        rr = np.concatenate([np.repeat(r, len(c)) for r, c, _ in blocks])
        cc = np.concatenate([np.tile(c, len(r)) for r, c, _ in blocks])
        vv = np.concatenate([b.ravel() for _, _, b in blocks])
        keep = vv != 0.0
        K = sps.csc_matrix((vv[keep], (rr[keep], cc[keep])), shape=(n_unk, n_unk))
        return K, layout
    K = np.zeros((n_unk, n_unk))
    for r, c, b in blocks:
        K[np.ix_(r, c)] = b
    return K, layout


def _panel_points(tree: Tree, disc: LeafDisc, i: int, f: int):
    pts = tree.leaf_boundary_points(disc, i)
    return pts[f * disc.n_face:(f + 1) * disc.n_face]


def rhs(tree: Tree, layout, f_src: np.ndarray | None, g_fun):
    """Right-hand side for sources f_src[leaf, point] and boundary values given
    by g_fun(points[..., d]) -> values."""
    disc = layout["disc"]
    n_unk = layout["n_u"] + len(layout["panels"]) * layout["nf"]
    b = np.zeros(n_unk)
    row = 0
    for i in range(tree.n_leaves):
        if f_src is not None:
            b[row:row + disc.n_i] = f_src[i][disc.Ii]
        row += disc.n_i + disc.n_e
    for key, r in layout["bnd_rows"].items():
        (i, f), = layout["owners"][key]
        b[r:r + layout["nf"]] = g_fun(_panel_points(tree, disc, i, f))
    return b


def solve(tree: Tree, p: int, coeffs, f_src, g_fun):
    K, layout = assemble(tree, p, coeffs)
    x = np.linalg.solve(K, rhs(tree, layout, f_src, g_fun))
    return x[:layout["n_u"]].reshape(tree.n_leaves, p ** tree.d)


def root_dtn(tree: Tree, p: int, coeffs, g_fun):
    """Outward normal derivative (Q u) on the root-boundary panels for f = 0
    and boundary data g_fun, keyed by panel, plus the points of each panel."""
    u = solve(tree, p, coeffs, None, g_fun)
    disc = LeafDisc(tree.d, p)
    Qr = disc.Q / tree.leaf_r
    nf = disc.n_face
    K, layout = assemble(tree, p, coeffs)
    out = []
    for key, r in layout["bnd_rows"].items():
        (i, f), = layout["owners"][key]
        out.append((_panel_points(tree, disc, i, f), (Qr @ u[i])[f * nf:(f + 1) * nf]))
    return out
