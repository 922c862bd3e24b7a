"""Plain CPU oracle of the HPS fast direct solver (DtN variant), fp64.

Test infrastructure only (see the package docstring).  It follows the paper's
algorithms step by step:

* Section 3.1 / Appendix A.1 / Appendix C.1: leaf discretization (Chebyshev--
  Lobatto tensor grid, Gauss--Legendre boundary panels with q = p - 2, the
  precomputed interpolation operator P and the normal-derivative operator Q).
* Algorithm "2D DtN local solve" (Appendix A.1, reused in 3D per Appendix C.1):
  Y = [I; -L_ii^{-1} L_ie] P,  v = [0; L_ii^{-1} f_i],  T = Q Y,  h = Q v.
* Algorithm "Merge stage" with eq. (merge_lin_system) and the Schur complement
  outputs of eqs. (merge_outputs_1, merge_outputs_2):
  T = A - B D^{-1} C,  h = h_ext - B D^{-1} h_int,  S = -D^{-1} C,
  g~ = -D^{-1} h_int; the blocks A, B, C, D, h_ext, h_int are those of
  Appendix A.2 (2D, written out literally below) and Appendix C.2 (3D).
* Algorithm "Downward pass": g_int = S g + g~, children data cut from
  [g_ext; g_int], and u = Y g + v at the leaves.
* The particular/homogeneous split of Section 3 lets sources enter at solve
  time: a build without f followed by a linear upward pass of h and g~.

Conventions this oracle fixes where the paper is silent (each is listed with
its reason in the design notes of the repository):

* leaf point order j = ix + p*iy (+ p^2*iz), nodes ascending;
* leaf boundary order: faces x-, x+, y-, y+, z-, z+ in 3D; sides S, E, N, W in
  2D; within a face the Gauss points in tensor order of the tangential
  coordinates (y,z), (x,z), (x,y) (first fastest); a parent face is the
  concatenation of its child faces in quadrant order (lo,lo), (hi,lo),
  (hi,hi), (lo,hi) of the tangential coordinates;
* children a, b, c, d = SW, SE, NE, NW (figure of the 2D merge); in 3D e..h
  lie directly above a..d;
* leaves are numbered depth-first (the children of a node are contiguous).
* the particular solution uses v_int = +L_ii^{-1} f_int so that L u = f holds
  on interior nodes (the printed algorithm carries a minus sign there, which
  would solve L u = -f).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.linalg as sla

from .spectral import cheb_lobatto, diff_matrix, gauss_legendre, interp_matrix

# --------------------------------------------------------------------------
# Geometry tables
# --------------------------------------------------------------------------
# face = (normal axis, side 0=lo / 1=hi, tangential axes)
FACES = {
    2: [(1, 0, (0,)), (0, 1, (1,)), (1, 1, (0,)), (0, 0, (1,))],          # S E N W
    3: [(0, 0, (1, 2)), (0, 1, (1, 2)), (1, 0, (0, 2)), (1, 1, (0, 2)),
        (2, 0, (0, 1)), (2, 1, (0, 1))],                                   # x- x+ y- y+ z- z+
}
# child offsets (per axis) in the order a, b, c, d (, e, f, g, h)
CHILD_OFFSETS = {
    2: [(0, 0), (1, 0), (1, 1), (0, 1)],
    3: [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0),
        (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)],
}
# quadrant order of sub-faces in (t1, t2): (lo,lo), (hi,lo), (hi,hi), (lo,hi)
QUADRANTS = [(0, 0), (1, 0), (1, 1), (0, 1)]
# interior interfaces of a merge, (child, face, child, face), in the paper's
# numbering 5..8 (2D) and 9..20 (3D)
INTERFACES = {
    2: [(0, 1, 1, 3),    # 5: a.E | b.W
        (1, 2, 2, 0),    # 6: b.N | c.S
        (2, 3, 3, 1),    # 7: c.W | d.E
        (3, 0, 0, 2)],   # 8: d.S | a.N
    3: [(0, 1, 1, 0), (1, 3, 2, 2), (2, 0, 3, 1), (3, 2, 0, 3),    # 9..12
        (4, 1, 5, 0), (5, 3, 6, 2), (6, 0, 7, 1), (7, 2, 4, 3),    # 13..16
        (0, 5, 4, 4), (1, 5, 5, 4), (2, 5, 6, 4), (3, 5, 7, 4)],   # 17..20
}


def n_terms(d):
    return 6 if d == 2 else 10


def face_children(d, f):
    """Children lying on parent face f, in the face's sub-face order."""
    axis, side, tang = FACES[d][f]
    out = []
    subs = [(0,), (1,)] if d == 2 else QUADRANTS
    for sub in subs:
        for c, off in enumerate(CHILD_OFFSETS[d]):
            if off[axis] != side:
                continue
            if all(off[t] == s for t, s in zip(tang, sub)):
                out.append(c)
    return out


def exterior_faces(d, c):
    """Faces of child c that lie on the parent's boundary, in face order."""
    off = CHILD_OFFSETS[d][c]
    return [f for f, (axis, side, _) in enumerate(FACES[d]) if off[axis] == side]


# --------------------------------------------------------------------------
# Leaf discretization (reference cell [-1, 1]^d)
# --------------------------------------------------------------------------
class LeafDisc:
    def __init__(self, d: int, p: int):
        self.d, self.p, self.q = d, p, p - 2
        q = self.q
        self.x = cheb_lobatto(p)
        self.D = diff_matrix(self.x)
        self.gl, self.glw = gauss_legendre(q)
        self.G2C = interp_matrix(self.gl, self.x)      # p x q
        self.C2G = interp_matrix(self.x, self.gl)      # q x p
        npts = p ** d
        idx = np.arange(npts)
        self.coords = np.stack([(idx // p ** a) % p for a in range(d)], axis=1)
        inner = np.all((self.coords >= 1) & (self.coords <= p - 2), axis=1)
        self.Ii = idx[inner]
        self.Ie = idx[~inner]
        self.n_i, self.n_e = len(self.Ii), len(self.Ie)
        self.n_face = q ** (d - 1)
        self.n_b = 2 * d * self.n_face
        # Chebyshev points of each face, tensor order of tangential coords
        self.face_cheb = []
        for axis, side, tang in FACES[d]:
            sel = self.coords[:, axis] == (0 if side == 0 else p - 1)
            pts = idx[sel]
            key = sum(self.coords[pts, t] * p ** k for k, t in enumerate(tang))
            self.face_cheb.append(pts[np.argsort(key)])
        # 1D -> face interpolation (Gauss <-> Chebyshev), tensor order t1 fastest
        if d == 2:
            g2c_face, c2g_face = self.G2C, self.C2G
        else:
            g2c_face = np.kron(self.G2C, self.G2C)
            c2g_face = np.kron(self.C2G, self.C2G)
        self.g2c_face, self.c2g_face = g2c_face, c2g_face
        # P: Gauss boundary data -> exterior Chebyshev points; a point on
        # several faces (corner / edge) averages their interpolants.
        pos_e = -np.ones(npts, dtype=int)
        pos_e[self.Ie] = np.arange(self.n_e)
        P = np.zeros((self.n_e, self.n_b))
        cnt = np.zeros(self.n_e)
        for f in range(2 * d):
            cols = slice(f * self.n_face, (f + 1) * self.n_face)
            for t, pt in enumerate(self.face_cheb[f]):
                P[pos_e[pt], cols] += g2c_face[t]
                cnt[pos_e[pt]] += 1
        self.P = P / cnt[:, None]
        # derivative matrices on the full tensor grid (reference cell)
        I = np.eye(p)
        self.Dax = []
        for a in range(d):
            mats = [I] * d
            mats[a] = self.D
            M = mats[d - 1]
            for k in range(d - 2, -1, -1):
                M = np.kron(M, mats[k])
            self.Dax.append(M)
        # Q: outward normal derivative at each face's Chebyshev points, then
        # Chebyshev -> Gauss interpolation on that face.
        Q = np.zeros((self.n_b, npts))
        for f, (axis, side, _) in enumerate(FACES[d]):
            sign = 1.0 if side == 1 else -1.0
            Nf = sign * self.Dax[axis][self.face_cheb[f], :]
            Q[f * self.n_face:(f + 1) * self.n_face] = c2g_face @ Nf
        self.Q = Q

    def term_ops(self, r: float):
        """Derivative operators of each coefficient term on a cell of
        half-width r, in the term order of the coefficient layout."""
        Dx = [M / r for M in self.Dax]
        I = np.eye(self.p ** self.d)
        if self.d == 2:
            x, y = Dx
            return [x @ x, x @ y, y @ y, x, y, I]
        x, y, z = Dx
        return [x @ x, y @ y, z @ z, x @ y, x @ z, y @ z, x, y, z, I]


# --------------------------------------------------------------------------
# Uniform tree over a cube
# --------------------------------------------------------------------------
class Tree:
    def __init__(self, d: int, depth: int, lo=-1.0, hi=1.0):
        self.d, self.L = d, depth
        self.lo, self.hi = float(lo), float(hi)
        self.n_leaves = 2 ** (d * depth)
        self.leaf_r = (self.hi - self.lo) / 2.0 / 2 ** depth

    def leaf_corner(self, i: int):
        """Lower corner of leaf i (depth-first numbering)."""
        corner = np.full(self.d, self.lo)
        size = self.hi - self.lo
        nd = 2 ** self.d
        digits = []
        for _ in range(self.L):
            digits.append(i % nd)
            i //= nd
        for c in reversed(digits):
            size /= 2.0
            corner = corner + size * np.array(CHILD_OFFSETS[self.d][c])
        return corner

    def leaf_points(self, disc: LeafDisc) -> np.ndarray:
        ref = disc.x[disc.coords]                                 # [np, d]
        out = np.empty((self.n_leaves, disc.p ** self.d, self.d))
        for i in range(self.n_leaves):
            out[i] = self.leaf_corner(i) + (ref + 1.0) * self.leaf_r
        return out

    def leaf_boundary_points(self, disc: LeafDisc, i: int) -> np.ndarray:
        """Gauss boundary points of leaf i in leaf boundary order."""
        corner, r = self.leaf_corner(i), self.leaf_r
        out = []
        g = disc.gl
        for axis, side, tang in FACES[self.d]:
            if len(tang) == 1:
                tvals = [g]
            else:  # tensor order, first tangential coordinate fastest
                tvals = [np.tile(g, len(g)), np.repeat(g, len(g))]
            pts = np.empty((len(tvals[0]), self.d))
            pts[:, axis] = corner[axis] + (2.0 * r if side == 1 else 0.0)
            for t, v in zip(tang, tvals):
                pts[:, t] = corner[t] + (v + 1.0) * r
            out.append(pts)
        return np.concatenate(out, axis=0)

    def root_boundary_points(self, disc: LeafDisc) -> np.ndarray:
        """Gauss points on the root boundary in root boundary order (parent
        faces are concatenations of child faces, recursively)."""
        nd = 2 ** self.d
        # boundary points per node, level by level from the leaves up
        level = [self.leaf_boundary_points(disc, i) for i in range(self.n_leaves)]
        nf = disc.n_face
        for _ in range(self.L):
            nxt = []
            for j in range(len(level) // nd):
                kids = level[nd * j: nd * j + nd]
                per_face = len(kids[0]) // (2 * self.d)
                faces = []
                for f in range(2 * self.d):
                    for c in face_children(self.d, f):
                        faces.append(kids[c][f * per_face:(f + 1) * per_face])
                nxt.append(np.concatenate(faces, axis=0))
            level = nxt
            nf *= 2 ** (self.d - 1)
        return level[0]


# --------------------------------------------------------------------------
# Leaf stage (Algorithm "2D DtN local solve"; Appendix C.1 in 3D)
# --------------------------------------------------------------------------
class Leaf:
    __slots__ = ("T", "h", "Y", "v", "lu")


def leaf_operator(disc: LeafDisc, ops, c: np.ndarray) -> np.ndarray:
    """L^(i) = sum_t diag(c_t) D_t on the leaf's p^d Chebyshev points."""
    L = np.zeros_like(ops[0])
    for t, Dt in enumerate(ops):
        L += c[t][:, None] * Dt
    return L


def leaf_solve(disc: LeafDisc, ops, Qr: np.ndarray, c: np.ndarray, f=None) -> Leaf:
    L = leaf_operator(disc, ops, c)
    Lii = L[np.ix_(disc.Ii, disc.Ii)]
    Lie = L[np.ix_(disc.Ii, disc.Ie)]
    lu = sla.lu_factor(Lii)                           # "Invert L(I_i, I_i)"
    npts = disc.p ** disc.d
    Y = np.zeros((npts, disc.n_b))
    Y[disc.Ie] = disc.P
    Y[disc.Ii] = -sla.lu_solve(lu, Lie) @ disc.P      # [I; -L_ii^{-1} L_ie] P
    v = np.zeros(npts)
    if f is not None:
        v[disc.Ii] = sla.lu_solve(lu, f[disc.Ii])     # particular solution
    out = Leaf()
    out.T = Qr @ Y
    out.h = Qr @ v
    out.Y, out.v, out.lu = Y, v, lu
    return out


# --------------------------------------------------------------------------
# Merge stage
# --------------------------------------------------------------------------
class MergeNode:
    __slots__ = ("S", "gt", "perm", "D_lu", "Dinv", "B", "ext_idx", "int_idx", "n", "cond1")


def _child_index_sets(d: int, n: int):
    """Per child: boundary indices of its exterior segment (exterior faces in
    face order) and of its face on each interior interface it touches."""
    nd = 2 ** d
    ext = [np.concatenate([np.arange(f * n, (f + 1) * n) for f in exterior_faces(d, c)])
           for c in range(nd)]
    inter = [dict() for _ in range(nd)]
    for i, (c1, f1, c2, f2) in enumerate(INTERFACES[d]):
        inter[c1][i] = np.arange(f1 * n, (f1 + 1) * n)
        inter[c2][i] = np.arange(f2 * n, (f2 + 1) * n)
    return ext, inter


def parent_order(d: int, n: int) -> np.ndarray:
    """perm[k] = position, in the exterior-segment order [seg 1; seg 2; ...],
    of the parent's k-th boundary point (parent boundary order)."""
    nd = 2 ** d
    seg_start, cur = [], 0
    for c in range(nd):
        seg_start.append(cur)
        cur += n * len(exterior_faces(d, c))
    perm = []
    for f in range(2 * d):
        for c in face_children(d, f):
            rank = exterior_faces(d, c).index(f)
            perm.append(seg_start[c] + rank * n + np.arange(n))
    return np.concatenate(perm)


def merge_blocks_2d(T, h, n):
    """Blocks of eq. (merge_lin_system) for the 2D four-to-one merge, written
    as in Appendix A.2 (children a, b, c, d; boundary segments 1..8)."""
    S_, E_, N_, W_ = 0, 1, 2, 3

    def side(s):
        return np.arange(s * n, (s + 1) * n)

    seg = [
        {1: np.concatenate([side(S_), side(W_)]), 5: side(E_), 8: side(N_)},   # a
        {2: np.concatenate([side(S_), side(E_)]), 5: side(W_), 6: side(N_)},   # b
        {3: np.concatenate([side(E_), side(N_)]), 6: side(S_), 7: side(W_)},   # c
        {4: np.concatenate([side(N_), side(W_)]), 7: side(E_), 8: side(S_)},   # d
    ]
    a, b, c, d = 0, 1, 2, 3

    def Tb(x, r, s):
        return T[x][np.ix_(seg[x][r], seg[x][s])]

    def hb(x, r):
        return h[x][seg[x][r]]

    Z2 = np.zeros((2 * n, n))
    Zt = np.zeros((n, 2 * n))
    Z1 = np.zeros((n, n))
    A = sla.block_diag(Tb(a, 1, 1), Tb(b, 2, 2), Tb(c, 3, 3), Tb(d, 4, 4))
    B = np.block([
        [Tb(a, 1, 5), Z2, Z2, Tb(a, 1, 8)],
        [Tb(b, 2, 5), Tb(b, 2, 6), Z2, Z2],
        [Z2, Tb(c, 3, 6), Tb(c, 3, 7), Z2],
        [Z2, Z2, Tb(d, 4, 7), Tb(d, 4, 8)],
    ])
    C = np.block([
        [Tb(a, 5, 1), Tb(b, 5, 2), Zt, Zt],
        [Zt, Tb(b, 6, 2), Tb(c, 6, 3), Zt],
        [Zt, Zt, Tb(c, 7, 3), Tb(d, 7, 4)],
        [Tb(a, 8, 1), Zt, Zt, Tb(d, 8, 4)],
    ])
    D = np.block([
        [Tb(a, 5, 5) + Tb(b, 5, 5), Tb(b, 5, 6), Z1, Tb(a, 5, 8)],
        [Tb(b, 6, 5), Tb(b, 6, 6) + Tb(c, 6, 6), Tb(c, 6, 7), Z1],
        [Z1, Tb(c, 7, 6), Tb(c, 7, 7) + Tb(d, 7, 7), Tb(d, 7, 8)],
        [Tb(a, 8, 5), Z1, Tb(d, 8, 7), Tb(d, 8, 8) + Tb(a, 8, 8)],
    ])
    h_ext = np.concatenate([hb(a, 1), hb(b, 2), hb(c, 3), hb(d, 4)])
    h_int = np.concatenate([hb(a, 5) + hb(b, 5), hb(b, 6) + hb(c, 6),
                            hb(c, 7) + hb(d, 7), hb(d, 8) + hb(a, 8)])
    return A, B, C, D, h_ext, h_int


def merge_blocks_general(d, T, h, n):
    """Blocks of eq. (merge_lin_system) for any dimension: A is block diagonal
    over the children's exterior segments, B (C) couples a child's exterior
    segment to (from) each interface it touches, and D sums, over the children
    touching two interfaces, their DtN blocks between them.  For d = 3 this is
    the block pattern printed in Appendix C.2 (pinned in the tests against the
    printed pattern); for d = 2 it equals Appendix A.2."""
    nd = 2 ** d
    ext, inter = _child_index_sets(d, n)
    nI = len(INTERFACES[d])
    ext_sizes = [len(e) for e in ext]
    Ablocks = [T[c][np.ix_(ext[c], ext[c])] for c in range(nd)]
    A = sla.block_diag(*Ablocks)
    B = np.zeros((sum(ext_sizes), nI * n))
    C = np.zeros((nI * n, sum(ext_sizes)))
    D = np.zeros((nI * n, nI * n))
    h_int = np.zeros(nI * n)
    off = np.cumsum([0] + ext_sizes)
    for c in range(nd):
        for i, ii in inter[c].items():
            B[off[c]:off[c + 1], i * n:(i + 1) * n] = T[c][np.ix_(ext[c], ii)]
            C[i * n:(i + 1) * n, off[c]:off[c + 1]] = T[c][np.ix_(ii, ext[c])]
            h_int[i * n:(i + 1) * n] += h[c][ii]
            for j, jj in inter[c].items():
                D[i * n:(i + 1) * n, j * n:(j + 1) * n] += T[c][np.ix_(ii, jj)]
    h_ext = np.concatenate([h[c][ext[c]] for c in range(nd)])
    return A, B, C, D, h_ext, h_int


def merge(d, T, h, n, with_T=True, d_inverse="lu"):
    """One merge (Algorithm "Merge stage", inner loop body).  Returns the node
    record and the parent's T, h in parent boundary order.

    "Invert D" is read as an LU factorization with partial pivoting applied
    by triangular solves (d_inverse="lu", the default), or as the explicit
    inverse D^{-1} applied by products (d_inverse="explicit"); the algorithm
    does not say which, and the two differ only by rounding."""
    if d == 2:
        A, B, C, D, h_ext, h_int = merge_blocks_2d(T, h, n)
    else:
        A, B, C, D, h_ext, h_int = merge_blocks_general(d, T, h, n)
    D_lu, Dinv = None, None
    if d_inverse == "lu":
        D_lu = sla.lu_factor(D)                   # "Invert D"
        # reciprocal 1-norm condition estimate of D from its LU factors
        # (LAPACK gecon): DtN merges of Helmholtz operators can be ill
        # conditioned near interior resonances (Section 2, related work)
        rcond1 = sla.lapack.dgecon(D_lu[0], np.linalg.norm(D, 1), norm="1")[0]
        S = -sla.lu_solve(D_lu, C)                # S = -D^{-1} C
        gt = -sla.lu_solve(D_lu, h_int)           # g~ = -D^{-1} h_int
    elif d_inverse == "explicit":
        Dinv = sla.inv(D)                         # "Invert D", explicitly
        S = -(Dinv @ C)
        gt = -(Dinv @ h_int)
    else:
        raise ValueError(d_inverse)
    h_seg = h_ext + B @ gt                        # h = h_ext - B D^{-1} h_int
    perm = parent_order(d, n)
    node = MergeNode()
    node.S, node.gt, node.perm, node.D_lu, node.Dinv, node.B, node.n = S, gt, perm, D_lu, Dinv, B, n
    node.cond1 = (1.0 / rcond1 if rcond1 > 0 else np.inf) if d_inverse == "lu" else np.linalg.cond(D, 1)
    Tp = None
    if with_T:
        T_seg = A + B @ S                         # T = A - B D^{-1} C
        Tp = T_seg[np.ix_(perm, perm)]
    return node, Tp, h_seg[perm]


# --------------------------------------------------------------------------
# Whole build / solve
# --------------------------------------------------------------------------
class Operator:
    pass


def build(tree: Tree, p: int, coeffs: np.ndarray, f: np.ndarray | None = None,
          root_T: bool = False, d_inverse: str = "lu") -> Operator:
    """Local solve stage + merge stage.  coeffs[leaf, term, point]; f (optional)
    [leaf, point] folds a source into the build (paper form); d_inverse
    selects the reading of "Invert D" (see merge)."""
    d = tree.d
    disc = LeafDisc(d, p)
    ops = disc.term_ops(tree.leaf_r)
    Qr = disc.Q / tree.leaf_r
    leaves = [leaf_solve(disc, ops, Qr, coeffs[i], None if f is None else f[i])
              for i in range(tree.n_leaves)]
    T = [lf.T for lf in leaves]
    h = [lf.h for lf in leaves]
    nd = 2 ** d
    n = disc.n_face
    levels = []
    for lev in range(tree.L - 1, -1, -1):
        nodes, Tn, hn = [], [], []
        for j in range(len(T) // nd):
            kids = slice(nd * j, nd * j + nd)
            node, Tp, hp = merge(d, T[kids], h[kids], n, with_T=(lev > 0 or root_T), d_inverse=d_inverse)
            nodes.append(node)
            Tn.append(Tp)
            hn.append(hp)
        levels.append(nodes)
        T, h = Tn, hn
        n *= 2 ** (d - 1)
    op = Operator()
    op.tree, op.p, op.disc, op.leaves = tree, p, disc, leaves
    op.levels = levels[::-1]          # levels[0] = root merge
    op.root_T, op.root_h = T[0], h[0]
    op.Qr = Qr
    return op


def _children_g(d, node: MergeNode, g_parent: np.ndarray, g_int: np.ndarray):
    n = node.n
    nd = 2 ** d
    g_ext = np.empty_like(g_parent)
    g_ext[node.perm] = g_parent
    ext, inter = _child_index_sets(d, n)
    off = np.cumsum([0] + [len(e) for e in ext])
    out = []
    for c in range(nd):
        gc = np.empty(2 * d * n)
        gc[ext[c]] = g_ext[off[c]:off[c + 1]]
        for i, ii in inter[c].items():
            gc[ii] = g_int[i * n:(i + 1) * n]
        out.append(gc)
    return out


def down_pass(op: Operator, g_root: np.ndarray, gt_levels=None, v_leaves=None):
    """Algorithm "Downward pass".  gt_levels / v_leaves override the stored
    particular data (used by the source-split solve)."""
    d = op.tree.d
    nd = 2 ** d
    g = [g_root]
    for lev, nodes in enumerate(op.levels):
        nxt = []
        for j, node in enumerate(nodes):
            gt = node.gt if gt_levels is None else gt_levels[lev][j]
            g_int = node.S @ g_ext_of(node, g[j]) + gt
            nxt.extend(_children_g(d, node, g[j], g_int))
        g = nxt
    u = np.empty((op.tree.n_leaves, op.p ** d))
    for i, lf in enumerate(op.leaves):
        v = lf.v if v_leaves is None else v_leaves[i]
        u[i] = lf.Y @ g[i] + v
    return u


def g_ext_of(node: MergeNode, g_parent: np.ndarray) -> np.ndarray:
    g_ext = np.empty_like(g_parent)
    g_ext[node.perm] = g_parent
    return g_ext


def up_pass(op: Operator, f: np.ndarray):
    """Linear upward pass of a source given at solve time (particular /
    homogeneous split): leaf v, h = Q v; per merge g~ = -D^{-1} h_int and
    h = h_ext + B g~ (the h, g~ formulas of eqs. merge_outputs_1/2)."""
    d = op.tree.d
    disc = op.disc
    nd = 2 ** d
    v_leaves, h = [], []
    for i, lf in enumerate(op.leaves):
        v = np.zeros(op.p ** d)
        v[disc.Ii] = sla.lu_solve(lf.lu, f[i][disc.Ii])
        v_leaves.append(v)
        h.append(op.Qr @ v)
    gt_levels = [None] * len(op.levels)
    for lev in range(len(op.levels) - 1, -1, -1):
        nodes = op.levels[lev]
        gts, hn = [], []
        for j, node in enumerate(nodes):
            n = node.n
            ext, inter = _child_index_sets(d, n)
            kids = h[nd * j: nd * j + nd]
            h_ext = np.concatenate([kids[c][ext[c]] for c in range(nd)])
            h_int = np.zeros(len(INTERFACES[d]) * n)
            for c in range(nd):
                for i, ii in inter[c].items():
                    h_int[i * n:(i + 1) * n] += kids[c][ii]
            gt = -sla.lu_solve(node.D_lu, h_int) if node.Dinv is None else -(node.Dinv @ h_int)
            gts.append(gt)
            hn.append((h_ext + node.B @ gt)[node.perm])
        gt_levels[lev] = gts
        h = hn
    return gt_levels, v_leaves


def solve(op: Operator, g_root: np.ndarray, f: np.ndarray | None = None) -> np.ndarray:
    """u on every leaf point, [leaf, point].  With f given, the source enters
    through the linear upward pass; with f None, the particular data stored
    by the build (if any) is used."""
    if f is None:
        return down_pass(op, g_root)
    gt_levels, v_leaves = up_pass(op, f)
    return down_pass(op, g_root, gt_levels, v_leaves)


def merge_sizes(d: int, p: int, depth: int):
    """(#merges, size of D, size of the parent T) per level, leaves upward."""
    q = p - 2
    n = q ** (d - 1)
    out = []
    for lev in range(depth - 1, -1, -1):
        nI = len(INTERFACES[d])
        nmerge = 2 ** (d * lev)
        out.append((nmerge, nI * n, 2 * d * n * 2 ** (d - 1)))
        n *= 2 ** (d - 1)
    return out
