"""Plain CPU oracle of the ItI (impedance-to-impedance) variant of the 2D HPS
method, complex128.  Test infrastructure only (see the package docstring).

It follows Appendix B ("Full algorithms for 2D problems using ItI matrices")
step by step:

* impedance data (Section 2): incoming g = u_n + i eta u, outgoing
  h = u_n - i eta u, eta > 0;
* leaf precomputation (Appendix B.1): P (Gauss -> the 4p - 4 boundary
  Chebyshev points, one interpolation block per side with one end row
  deleted), Q (Chebyshev -> Gauss per side, corners counted twice),
  N~ / G = N~ + i eta I (incoming impedance at the 4p - 4 boundary points),
  N / H = N - i eta I (outgoing impedance at the 4p points, corners twice);
* Algorithm "2D ItI local solve": B = [G; L(I_i, :)], Y = B^{-1}(:, I_e) P,
  v = B^{-1}(:, I_i) f(I_i), T = Q H Y, h = Q H v (B^{-1} applied through its
  LU factors);
* the merge of Appendix B.2: constraints eq. (2D_ItI_merge_1) and
  eq. (2D_ItI_merge_2) with the blocks A, B, C, D, h_ext, h_int written out
  literally as printed, and D^{-1} from the Schur complement
  W = I - D_12 D_21 of eq. (ItI_D_inv);
* outputs by eqs. (merge_outputs_1, merge_outputs_2):
  S = -D^{-1} C, T = A + B S, g~ = -D^{-1} h_int, h = h_ext + B g~;
* the downward pass of the DtN variant with incoming impedance data in
  place of Dirichlet data, and u = Y g + v at the leaves; sources enter at
  solve time through the linear upward pass (particular / homogeneous split,
  Section 3), exactly as in the DtN oracle.

Conventions fixed here where the paper is silent (listed with their reasons
in the design notes of the repository):

* points, sides (S, E, N, W, points in ascending tangential coordinate),
  children (a, b, c, d = SW, SE, NE, NW) and the root boundary order are
  those of the DtN oracle (``oracle.hps``);
* "the final row deleted" per side is read along a counterclockwise walk of
  the boundary: every corner carries the Robin condition of the side that
  starts at it (SW -> S, SE -> E, NE -> N, NW -> W); in ascending order S and
  E keep their first p - 1 points, N and W their last p - 1;
* the rows of B are the 4p - 4 Robin rows (sides in order, points ascending)
  followed by the interior rows in ascending point index, so B^{-1}(:, I_e)
  and B^{-1}(:, I_i) are its first 4p - 4 and last (p - 2)^2 columns.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .hps import FACES, LeafDisc, Tree, parent_order

__all__ = ["ItiLeafOps", "leaf_solve", "merge", "build", "up_pass", "solve", "robin_rows"]

S_, E_, N_, W_ = 0, 1, 2, 3


def robin_rows(disc: LeafDisc):
    """(point, side, position along the side) of the 4p - 4 Robin rows."""
    p = disc.p
    rows = []
    for f in range(4):
        pts = disc.face_cheb[f]
        ts = range(0, p - 1) if f in (S_, E_) else range(1, p)
        for t in ts:
            rows.append((int(pts[t]), f, t))
    return rows


class ItiLeafOps:
    """The precomputed leaf matrices of Appendix B.1 on a leaf of half-width
    r, with impedance parameter eta."""

    def __init__(self, disc: LeafDisc, r: float, eta: float):
        p, q = disc.p, disc.q
        self.disc, self.r, self.eta = disc, r, eta
        npts = p * p
        Dx = [M / r for M in disc.Dax]

        def normal_row(pt, f):
            axis, side, _ = FACES[2][f]
            return (1.0 if side == 1 else -1.0) * Dx[axis][pt]

        rows = robin_rows(disc)
        self.n_r = len(rows)                                   # 4p - 4
        G = np.zeros((self.n_r, npts), dtype=complex)
        P = np.zeros((self.n_r, 4 * q))
        for k, (pt, f, t) in enumerate(rows):
            G[k] = normal_row(pt, f)                          # N~
            G[k, pt] += 1j * eta                              # + i eta I
            P[k, f * q:(f + 1) * q] = disc.G2C[t]
        H = np.zeros((4 * p, npts), dtype=complex)
        Q = np.zeros((4 * q, 4 * p))
        for f in range(4):
            for t, pt in enumerate(disc.face_cheb[f]):
                H[f * p + t] = normal_row(pt, f)              # N
                H[f * p + t, pt] -= 1j * eta                  # - i eta I
            Q[f * q:(f + 1) * q, f * p:(f + 1) * p] = disc.C2G
        self.G, self.P, self.H, self.Q = G, P, H, Q
        self.QH = Q @ H
        self.terms = disc.term_ops(r)


class Leaf:
    __slots__ = ("T", "h", "Y", "v", "lu")


def leaf_solve(ops: ItiLeafOps, c: np.ndarray, f=None) -> Leaf:
    """Algorithm "2D ItI local solve" for one leaf with coefficients c[term, pt]."""
    disc = ops.disc
    npts = disc.p ** 2
    L = np.zeros((npts, npts), dtype=complex)
    for t, Dt in enumerate(ops.terms):
        L += c[t][:, None] * Dt
    B = np.vstack([ops.G, L[disc.Ii]])
    lu = sla.lu_factor(B)                                     # "Invert B"
    rhs = np.zeros((npts, ops.P.shape[1]), dtype=complex)
    rhs[:ops.n_r] = ops.P
    Y = sla.lu_solve(lu, rhs)                                 # B^{-1}(:, I_e) P
    v = np.zeros(npts, dtype=complex)
    if f is not None:
        b = np.zeros(npts, dtype=complex)
        b[ops.n_r:] = f[disc.Ii]
        v = sla.lu_solve(lu, b)                               # B^{-1}(:, I_i) f(I_i)
    out = Leaf()
    out.T = ops.QH @ Y
    out.h = ops.QH @ v
    out.Y, out.v, out.lu = Y, v, lu
    return out


class MergeNode:
    __slots__ = ("S", "Dinv", "B", "gt", "perm", "n")


def _segments(n):
    """Per child a, b, c, d: boundary indices of its exterior part (1..4)
    and of its sides on the interfaces 5..8."""
    def side(s):
        return np.arange(s * n, (s + 1) * n)

    return [
        {1: np.concatenate([side(S_), side(W_)]), 5: side(E_), 8: side(N_)},   # a
        {2: np.concatenate([side(S_), side(E_)]), 5: side(W_), 6: side(N_)},   # b
        {3: np.concatenate([side(E_), side(N_)]), 6: side(S_), 7: side(W_)},   # c
        {4: np.concatenate([side(N_), side(W_)]), 7: side(E_), 8: side(S_)},   # d
    ]


def h_blocks(h, n):
    """h_ext and h_int of Appendix B.2 (h_int in the order of the constraint
    rows: the outgoing data of the neighbour across each unknown's side)."""
    seg = _segments(n)
    a, b, c, d = 0, 1, 2, 3

    def hb(x, r):
        return h[x][seg[x][r]]

    h_ext = np.concatenate([hb(a, 1), hb(b, 2), hb(c, 3), hb(d, 4)])
    h_int = np.concatenate([hb(b, 5), hb(d, 8), hb(b, 6), hb(d, 7),
                            hb(a, 5), hb(c, 6), hb(c, 7), hb(a, 8)])
    return h_ext, h_int


def merge_blocks(T, h, n):
    """A, B, C, D, h_ext, h_int of Appendix B.2 for children a, b, c, d and
    boundary parts 1..8 (parts 1-4: the children's exterior sides; 5-8: the
    interfaces a|b, b|c, c|d, d|a), with
    g_int = [g5a, g8a, g6c, g7c, g5b, g6b, g7d, g8d]."""
    seg = _segments(n)
    a, b, c, d = 0, 1, 2, 3

    def Tb(x, r, s):
        return T[x][np.ix_(seg[x][r], seg[x][s])]

    Z1 = np.zeros((n, n), dtype=complex)
    Z2 = np.zeros((2 * n, n), dtype=complex)
    Zt = np.zeros((n, 2 * n), dtype=complex)
    A = sla.block_diag(Tb(a, 1, 1), Tb(b, 2, 2), Tb(c, 3, 3), Tb(d, 4, 4))
    B = np.block([
        [Tb(a, 1, 5), Tb(a, 1, 8), Z2, Z2, Z2, Z2, Z2, Z2],
        [Z2, Z2, Z2, Z2, Tb(b, 2, 5), Tb(b, 2, 6), Z2, Z2],
        [Z2, Z2, Tb(c, 3, 6), Tb(c, 3, 7), Z2, Z2, Z2, Z2],
        [Z2, Z2, Z2, Z2, Z2, Z2, Tb(d, 4, 7), Tb(d, 4, 8)],
    ])
    C = np.block([
        [Zt, Tb(b, 5, 2), Zt, Zt],
        [Zt, Zt, Zt, Tb(d, 8, 4)],
        [Zt, Tb(b, 6, 2), Zt, Zt],
        [Zt, Zt, Zt, Tb(d, 7, 4)],
        [Tb(a, 5, 1), Zt, Zt, Zt],
        [Zt, Zt, Tb(c, 6, 3), Zt],
        [Zt, Zt, Tb(c, 7, 3), Zt],
        [Tb(a, 8, 1), Zt, Zt, Zt],
    ])
    D = np.eye(8 * n, dtype=complex) + np.block([
        [Z1, Z1, Z1, Z1, Tb(b, 5, 5), Tb(b, 5, 6), Z1, Z1],
        [Z1, Z1, Z1, Z1, Z1, Z1, Tb(d, 8, 7), Tb(d, 8, 8)],
        [Z1, Z1, Z1, Z1, Tb(b, 6, 5), Tb(b, 6, 6), Z1, Z1],
        [Z1, Z1, Z1, Z1, Z1, Z1, Tb(d, 7, 7), Tb(d, 7, 8)],
        [Tb(a, 5, 5), Tb(a, 5, 8), Z1, Z1, Z1, Z1, Z1, Z1],
        [Z1, Z1, Tb(c, 6, 6), Tb(c, 6, 7), Z1, Z1, Z1, Z1],
        [Z1, Z1, Tb(c, 7, 6), Tb(c, 7, 7), Z1, Z1, Z1, Z1],
        [Tb(a, 8, 5), Tb(a, 8, 8), Z1, Z1, Z1, Z1, Z1, Z1],
    ])
    h_ext, h_int = h_blocks(h, n)
    return A, B, C, D, h_ext, h_int


def d_inverse(D: np.ndarray, n: int) -> np.ndarray:
    """D^{-1} by eq. (ItI_D_inv): D = [[I, D12], [D21, I]], W = I - D12 D21,
    D^{-1} = [[W^{-1}, -W^{-1} D12], [-D21 W^{-1}, I + D21 W^{-1} D12]]."""
    k = 4 * n
    D12, D21 = D[:k, k:], D[k:, :k]
    W = np.eye(k) - D12 @ D21
    Winv = sla.inv(W)                                          # the one inversion
    return np.block([[Winv, -Winv @ D12],
                     [-D21 @ Winv, np.eye(k) + D21 @ Winv @ D12]])


def merge(T, h, n, with_T=True):
    A, B, C, D, h_ext, h_int = merge_blocks(T, h, n)
    Dinv = d_inverse(D, n)
    S = -(Dinv @ C)
    gt = -(Dinv @ h_int)
    perm = parent_order(2, n)
    node = MergeNode()
    node.S, node.Dinv, node.B, node.gt, node.perm, node.n = S, Dinv, B, gt, perm, n
    Tp = (A + B @ S)[np.ix_(perm, perm)] if with_T else None
    return node, Tp, (h_ext + B @ gt)[perm]


class Operator:
    pass


def build(tree: Tree, p: int, eta: float, coeffs: np.ndarray, f=None) -> Operator:
    """Local solve stage + merge stage of the ItI variant (2D).  coeffs[leaf,
    term, point] (real or complex); f (optional) folds a source into the
    build (paper form)."""
    assert tree.d == 2
    disc = LeafDisc(2, p)
    ops = ItiLeafOps(disc, tree.leaf_r, eta)
    leaves = [leaf_solve(ops, coeffs[i], None if f is None else f[i]) for i in range(tree.n_leaves)]
    T = [lf.T for lf in leaves]
    h = [lf.h for lf in leaves]
    n = disc.q
    levels = []
    for lev in range(tree.L - 1, -1, -1):
        nodes, Tn, hn = [], [], []
        for j in range(len(T) // 4):
            node, Tp, hp = merge(T[4 * j:4 * j + 4], h[4 * j:4 * j + 4], n, with_T=lev > 0)
            nodes.append(node)
            Tn.append(Tp)
            hn.append(hp)
        levels.append(nodes)
        T, h = Tn, hn
        n *= 2
    op = Operator()
    op.tree, op.p, op.eta, op.disc, op.ops, op.leaves = tree, p, eta, disc, ops, leaves
    op.levels = levels[::-1]
    op.root_h = h[0]
    return op


def _children_g(node: MergeNode, g_parent, g_int):
    """Incoming data of the four children: exterior sides from the parent,
    interface sides from g_int = [g5a, g8a, g6c, g7c, g5b, g6b, g7d, g8d]."""
    n = node.n
    g_ext = np.empty_like(g_parent)
    g_ext[node.perm] = g_parent
    part = [g_ext[k * 2 * n:(k + 1) * 2 * n] for k in range(4)]
    gi = [g_int[k * n:(k + 1) * n] for k in range(8)]
    out = []
    for c, (ext_sides, ints) in enumerate([
            ((S_, W_), ((E_, 0), (N_, 1))),     # a: g5a on E, g8a on N
            ((S_, E_), ((W_, 4), (N_, 5))),     # b: g5b on W, g6b on N
            ((E_, N_), ((S_, 2), (W_, 3))),     # c: g6c on S, g7c on W
            ((N_, W_), ((E_, 6), (S_, 7)))]):   # d: g7d on E, g8d on S
        g = np.empty(4 * n, dtype=complex)
        for k, s in enumerate(ext_sides):
            g[s * n:(s + 1) * n] = part[c][k * n:(k + 1) * n]
        for s, k in ints:
            g[s * n:(s + 1) * n] = gi[k]
        out.append(g)
    return out


def up_pass(op: Operator, f: np.ndarray):
    """Linear upward pass of a source given at solve time: leaf v and h; per
    merge g~ = -D^{-1} h_int and h = h_ext + B g~."""
    disc, ops = op.disc, op.ops
    v_leaves, h = [], []
    for i, lf in enumerate(op.leaves):
        b = np.zeros(disc.p ** 2, dtype=complex)
        b[ops.n_r:] = f[i][disc.Ii]
        v = sla.lu_solve(lf.lu, b)
        v_leaves.append(v)
        h.append(ops.QH @ v)
    gt_levels = [None] * len(op.levels)
    for lev in range(len(op.levels) - 1, -1, -1):
        gts, hn = [], []
        for j, node in enumerate(op.levels[lev]):
            h_ext, h_int = h_blocks(h[4 * j:4 * j + 4], node.n)
            gt = -(node.Dinv @ h_int)
            gts.append(gt)
            hn.append((h_ext + node.B @ gt)[node.perm])
        gt_levels[lev] = gts
        h = hn
    return gt_levels, v_leaves


def solve(op: Operator, g_root: np.ndarray, f: np.ndarray | None = None) -> np.ndarray:
    """u at every leaf point [leaf, point] from the incoming impedance data
    g_root at the root's Gauss points (root boundary order) and a source f
    [leaf, point] (None: f = 0, or the source folded into the build)."""
    if f is not None:
        gt_levels, v_leaves = up_pass(op, f)
    else:
        gt_levels, v_leaves = None, None
    g = [np.asarray(g_root, dtype=complex)]
    for lev, nodes in enumerate(op.levels):
        nxt = []
        for j, node in enumerate(nodes):
            gt = node.gt if gt_levels is None else gt_levels[lev][j]
            g_ext = np.empty_like(g[j])
            g_ext[node.perm] = g[j]
            nxt.extend(_children_g(node, g[j], node.S @ g_ext + gt))
        g = nxt
    u = np.empty((op.tree.n_leaves, op.p ** 2), dtype=complex)
    for i, lf in enumerate(op.leaves):
        u[i] = lf.Y @ g[i] + (lf.v if v_leaves is None else v_leaves[i])
    return u
