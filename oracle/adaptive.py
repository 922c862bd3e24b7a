"""Adaptive 3D HPS (Section 4.2), fp64 -- test infrastructure only.

Plain NumPy/SciPy, written from the paper's description of the adaptive
discretization (see the package docstring for who may import this module):

* Refinement criterion, eq. (refinement_check): a leaf is refined enough for
  a function f when the interpolant through its p^3 Chebyshev samples x_0
  reproduces f at the 8 p^3 Chebyshev points x_1 of its eight children,
  || f(x_1) - L_8f1 f(x_0) ||_inf < eps || f ||_inf.  A failing leaf is split
  into eight and its children are checked in turn.  One tree is refined per
  function (coefficients and source); the discretization tree is their union.
* Level restriction: leaves are split until no leaf has a face neighbour
  whose side is less than half its own (at most one level apart across every
  face), which is what makes every projection four-to-one.
* Local solves: the uniform leaf stage on every leaf, with the leaf's own
  half-width in the derivative operators and in Q.
* Non-uniform merges: the eight children keep their own exterior panels
  (the parent's boundary inherits them).  Each interior interface is
  discretized on the coarser of its two sides, panel by panel: where one side
  has one Gauss panel and the other the four panels of its quadrants, the
  fine side's Dirichlet data are the coarse panel's interpolant at the fine
  Gauss points (one-to-four interpolation, columns of B and D) and its
  Neumann data are interpolated from the four fine panels to the coarse Gauss
  points (four-to-one, rows of C, D and h_int).  Then the Schur complement
  outputs of eq. (merge_lin_system) as in the uniform merge.
* Downward pass: g_int = S g_ext + g~ on the coarse interface points; a fine
  child side receives the one-to-four interpolant of it.

Readings where the paper is silent (repeated in the design notes):
* the four-to-one operator evaluates, at each coarse Gauss point, the
  degree-(q-1) interpolant of the fine panel that contains it (a point on a
  quadrant boundary, possible only for odd q, is taken from the lower
  quadrant);
* || f ||_inf in the criterion is the largest |f| over the Chebyshev points
  of the current leaves of the tree being refined;
* the level restriction is across faces (the pairs the merges project
  between); edge and corner neighbours are not restricted;
* interface panels are ordered by a quadtree walk of the interface square,
  sub-squares in the same quadrant order as the sub-faces of a parent face,
  so that a uniform tree gives exactly the uniform merge.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .hps import CHILD_OFFSETS, FACES, INTERFACES, QUADRANTS, LeafDisc, exterior_faces, face_children, leaf_solve
from .spectral import gauss_legendre, interp_matrix

D3 = 3
ND = 8


# --------------------------------------------------------------------------
# Octree (nodes are (level, ix, iy, iz), integer corner at that level)
# --------------------------------------------------------------------------
def children(key):
    l, x, y, z = key
    return [(l + 1, 2 * x + o[0], 2 * y + o[1], 2 * z + o[2]) for o in CHILD_OFFSETS[D3]]


class AdaptiveTree:
    """Octree over the cube [lo, hi]^3 given by its set of leaves."""

    def __init__(self, leaves, lo=0.0, hi=1.0):
        self.lo, self.hi = float(lo), float(hi)
        self.leafset = set(leaves)
        internal = set()
        for (l, x, y, z) in self.leafset:
            while l > 0:
                l, x, y, z = l - 1, x // 2, y // 2, z // 2
                internal.add((l, x, y, z))
        self.internal = internal
        self.max_level = max(k[0] for k in self.leafset)
        # depth-first leaf order (children of a node contiguous)
        self.leaves = []

        def walk(k):
            if k in self.leafset:
                self.leaves.append(k)
            else:
                for c in children(k):
                    walk(c)

        walk((0, 0, 0, 0))
        assert len(self.leaves) == len(self.leafset), "leaves do not tile the cube"

    @staticmethod
    def uniform(depth, lo=0.0, hi=1.0):
        n = 2 ** depth
        return AdaptiveTree([(depth, x, y, z) for z in range(n) for y in range(n) for x in range(n)], lo, hi)

    def half_width(self, level):
        return (self.hi - self.lo) / 2.0 / 2 ** level

    def corner(self, key):
        l, x, y, z = key
        return self.lo + 2.0 * self.half_width(l) * np.array([x, y, z], dtype=float)

    def points(self, disc: LeafDisc, key):
        """Chebyshev points of a node's box in leaf point order."""
        r = self.half_width(key[0])
        return self.corner(key) + (disc.x[disc.coords] + 1.0) * r

    def leaf_points(self, disc: LeafDisc):
        return np.stack([self.points(disc, k) for k in self.leaves])

    def fine_box(self, key):
        """Integer box (lo, size) on the grid of the finest level."""
        l = key[0]
        s = 2 ** (self.max_level - l)
        return np.array(key[1:]) * s, s


# --------------------------------------------------------------------------
# Refinement criterion, union, level restriction
# --------------------------------------------------------------------------
def child_interp(p: int) -> np.ndarray:
    """L_8f1: values at a box's p^3 Chebyshev points -> values at the p^3
    Chebyshev points of each of its eight children (children in the merge's
    child order, each in leaf point order)."""
    disc = LeafDisc(D3, p)
    x = disc.x
    half = [interp_matrix(x, (x - 1.0) / 2.0), interp_matrix(x, (x + 1.0) / 2.0)]
    blocks = []
    for o in CHILD_OFFSETS[D3]:
        blocks.append(np.kron(half[o[2]], np.kron(half[o[1]], half[o[0]])))
    return np.vstack(blocks)


def refine_one(f, p: int, eps: float, max_level: int, lo=0.0, hi=1.0):
    """Leaves of the tree refined for one function f (callable on [N, 3])."""
    disc = LeafDisc(D3, p)
    L8 = child_interp(p)
    leaves = {(0, 0, 0, 0)}
    while True:
        t = AdaptiveTree(leaves, lo, hi)
        f0 = {k: f(t.points(disc, k)) for k in t.leaves}
        fnorm = max(np.max(np.abs(v)) for v in f0.values())
        split = []
        for k in t.leaves:
            if k[0] >= max_level or fnorm == 0.0:
                continue
            x1 = np.concatenate([t.points(disc, c) for c in children(k)])
            err = np.max(np.abs(f(x1) - L8 @ f0[k])) / fnorm
            if not err < eps:
                split.append(k)
        if not split:
            return leaves
        for k in split:
            leaves.remove(k)
            leaves.update(children(k))


def union(leafsets):
    """Leaves of the union of several trees: a node is split if any tree
    splits it."""
    internal = set()
    for ls in leafsets:
        for (l, x, y, z) in ls:
            while l > 0:
                l, x, y, z = l - 1, x // 2, y // 2, z // 2
                internal.add((l, x, y, z))
    out = set()
    for ls in leafsets:
        for k in ls:
            if k not in internal:
                out.add(k)
    # every child of an internal node is a node of the union
    for k in internal:
        for c in children(k):
            if c not in internal:
                out.add(c)
    return out


def face_neighbour_pairs(t: AdaptiveTree):
    """(i, j) over leaves i, j that share a face of positive area."""
    lo = np.array([t.fine_box(k)[0] for k in t.leaves])
    sz = np.array([t.fine_box(k)[1] for k in t.leaves])
    hi = lo + sz[:, None]
    pairs = []
    for i in range(len(t.leaves)):
        touch = np.zeros(len(t.leaves), dtype=bool)
        for a in range(3):
            o = [b for b in range(3) if b != a]
            contact = (hi[i, a] == lo[:, a]) | (hi[:, a] == lo[i, a])
            overlap = np.ones(len(t.leaves), dtype=bool)
            for b in o:
                overlap &= np.minimum(hi[i, b], hi[:, b]) > np.maximum(lo[i, b], lo[:, b])
            touch |= contact & overlap
        for j in np.nonzero(touch)[0]:
            pairs.append((i, int(j)))
    return pairs


def balance(leaves, lo=0.0, hi=1.0):
    """Split leaves until face neighbours differ by at most one level."""
    leaves = set(leaves)
    while True:
        t = AdaptiveTree(leaves, lo, hi)
        split = set()
        for i, j in face_neighbour_pairs(t):
            if t.leaves[j][0] >= t.leaves[i][0] + 2:
                split.add(t.leaves[i])
        if not split:
            return leaves
        for k in split:
            leaves.remove(k)
            leaves.update(children(k))


def adaptive_tree(funcs, p: int, eps: float, max_level: int, lo=0.0, hi=1.0) -> AdaptiveTree:
    """Section 4.2's tree: one refinement per function, union, level restriction."""
    trees = [refine_one(f, p, eps, max_level, lo, hi) for f in funcs]
    return AdaptiveTree(balance(union(trees), lo, hi), lo, hi)


def is_balanced(t: AdaptiveTree) -> bool:
    return all(abs(t.leaves[i][0] - t.leaves[j][0]) <= 1 for i, j in face_neighbour_pairs(t))


# --------------------------------------------------------------------------
# Gauss panels and the one-to-four / four-to-one operators
# --------------------------------------------------------------------------
def tangential(axis):
    return [b for b in range(3) if b != axis]


class Panels:
    """Panel operators for q Gauss points per side."""

    def __init__(self, q: int):
        self.q = q
        g, _ = gauss_legendre(q)
        self.g = g
        half = [interp_matrix(g, (g - 1.0) / 2.0), interp_matrix(g, (g + 1.0) / 2.0)]
        # one-to-four: coarse panel values -> Gauss values of sub-panel j
        self.up = [np.kron(half[s2], half[s1]) for (s1, s2) in QUADRANTS]
        # four-to-one: Gauss values of the four sub-panels -> coarse points
        q2 = q * q
        down = np.zeros((q2, 4 * q2))
        for b in range(q):
            for a in range(q):
                # the middle node of an odd rule lies on the seam (the
                # eigenvalue method leaves it within rounding of 0): lower quadrant
                s1, s2 = int(g[a] > 1e-12), int(g[b] > 1e-12)
                j = QUADRANTS.index((s1, s2))
                t1 = 2.0 * g[a] + (1.0 if s1 == 0 else -1.0)
                t2 = 2.0 * g[b] + (1.0 if s2 == 0 else -1.0)
                w1 = interp_matrix(g, np.array([t1]))[0]
                w2 = interp_matrix(g, np.array([t2]))[0]
                down[a + q * b, j * q2:(j + 1) * q2] = np.kron(w2, w1)
        self.down = down


def leaf_panels(t: AdaptiveTree, key):
    """The six faces of a leaf as (face, panel); panel = (axis, plane, t1lo,
    t2lo, size) on the finest-level integer grid."""
    lo, s = t.fine_box(key)
    out = []
    for f, (axis, side, tang) in enumerate(FACES[D3]):
        out.append((f, (axis, int(lo[axis] + side * s), int(lo[tang[0]]), int(lo[tang[1]]), int(s))))
    return out


def panel_points(t: AdaptiveTree, q: int, pan):
    """Gauss points of a panel, tangential tensor order (first fastest)."""
    axis, plane, a0, b0, s = pan
    g, _ = gauss_legendre(q)
    h = (t.hi - t.lo) / 2 ** t.max_level
    ta, tb = tangential(axis)
    pts = np.empty((q * q, 3))
    pts[:, axis] = t.lo + plane * h
    pts[:, ta] = t.lo + (a0 + (np.tile(g, q) + 1.0) * s / 2.0) * h
    pts[:, tb] = t.lo + (b0 + (np.repeat(g, q) + 1.0) * s / 2.0) * h
    return pts


# --------------------------------------------------------------------------
# Non-uniform merge
# --------------------------------------------------------------------------
class AdaptiveMerge:
    __slots__ = ("S", "gt", "D_lu", "B", "perm", "Ext", "Int", "Rint", "m", "ne", "nkids")


def coarse_squares(square, side1, side2):
    """Quadtree walk of an interface square: a square that is a panel of
    either side is an interface panel, otherwise its four quadrants are
    walked in quadrant order."""
    if square in side1 or square in side2:
        return [square]
    a0, b0, s = square
    h = s // 2
    if h == 0:
        raise ValueError("interface sides do not meet on common squares")
    out = []
    for (s1, s2) in QUADRANTS:
        out.extend(coarse_squares((a0 + s1 * h, b0 + s2 * h, h), side1, side2))
    return out


def merge_node(pan: Panels, kid_bdry, T, h):
    """One non-uniform merge.  kid_bdry[c] = child c's boundary as a list of
    (face, panel); T[c], h[c] on those points (q^2 per panel).  Returns the
    node record, the parent boundary, and the parent T and h (or None)."""
    q2 = pan.q * pan.q
    sizes = [len(b) * q2 for b in kid_bdry]
    # exterior segments, per child, in face order
    ext_panels = [[k for k, (f, _) in enumerate(kid_bdry[c]) if f in exterior_faces(D3, c)] for c in range(ND)]
    ne = sum(len(e) for e in ext_panels) * q2
    # interface discretizations
    iface = []
    m = 0
    for (c1, f1, c2, f2) in INTERFACES[D3]:
        s1 = {(p_[2], p_[3], p_[4]): k for k, (f, p_) in enumerate(kid_bdry[c1]) if f == f1}
        s2 = {(p_[2], p_[3], p_[4]): k for k, (f, p_) in enumerate(kid_bdry[c2]) if f == f2}
        a0 = min(k[0] for k in s1)
        b0 = min(k[1] for k in s1)
        size = max(k[0] + k[2] for k in s1) - a0
        sq = coarse_squares((a0, b0, size), s1, s2)
        iface.append((c1, s1, c2, s2, sq, m))
        m += len(sq) * q2
    Ext = [np.zeros((sizes[c], ne)) for c in range(ND)]
    Int = [np.zeros((sizes[c], m)) for c in range(ND)]
    Rint = [np.zeros((m, sizes[c])) for c in range(ND)]
    off = 0
    for c in range(ND):
        for k in ext_panels[c]:
            Ext[c][k * q2:(k + 1) * q2, off:off + q2] = np.eye(q2)
            off += q2
    for (c1, s1, c2, s2, sq, moff) in iface:
        for c, side in ((c1, s1), (c2, s2)):
            for j, (a0, b0, s) in enumerate(sq):
                o = moff + j * q2
                if (a0, b0, s) in side:
                    k = side[(a0, b0, s)]
                    Int[c][k * q2:(k + 1) * q2, o:o + q2] = np.eye(q2)
                    Rint[c][o:o + q2, k * q2:(k + 1) * q2] = np.eye(q2)
                    continue
                hs = s // 2
                for jj, (u1, u2) in enumerate(QUADRANTS):
                    sub = (a0 + u1 * hs, b0 + u2 * hs, hs)
                    if sub not in side:
                        raise ValueError("level restriction violated across an interface")
                    k = side[sub]
                    Int[c][k * q2:(k + 1) * q2, o:o + q2] = pan.up[jj]
                    Rint[c][o:o + q2, k * q2:(k + 1) * q2] = pan.down[:, jj * q2:(jj + 1) * q2]
    A = sum(Ext[c].T @ T[c] @ Ext[c] for c in range(ND))
    B = sum(Ext[c].T @ T[c] @ Int[c] for c in range(ND))
    C = sum(Rint[c] @ T[c] @ Ext[c] for c in range(ND))
    D = sum(Rint[c] @ T[c] @ Int[c] for c in range(ND))
    h_ext = sum(Ext[c].T @ h[c] for c in range(ND))
    h_int = sum(Rint[c] @ h[c] for c in range(ND))
    D_lu = sla.lu_factor(D)                       # "Invert D"
    S = -sla.lu_solve(D_lu, C)
    gt = -sla.lu_solve(D_lu, h_int)
    # parent boundary: faces in order, children on the face in sub-face order,
    # each child's panels on that face in its own order
    seg_pos = {}
    off = 0
    for c in range(ND):
        for k in ext_panels[c]:
            seg_pos[(c, k)] = off
            off += q2
    bdry, perm = [], []
    for f in range(2 * D3):
        for c in face_children(D3, f):
            for k, (ff, p_) in enumerate(kid_bdry[c]):
                if ff == f:
                    bdry.append((f, p_))
                    perm.append(seg_pos[(c, k)] + np.arange(q2))
    perm = np.concatenate(perm)
    node = AdaptiveMerge()
    node.S, node.gt, node.D_lu, node.B, node.perm = S, gt, D_lu, B, perm
    node.Ext, node.Int, node.Rint, node.m, node.ne, node.nkids = Ext, Int, Rint, m, ne, ND
    Tp = (A + B @ S)[np.ix_(perm, perm)]
    hp = (h_ext + B @ gt)[perm]
    return node, bdry, Tp, hp


# --------------------------------------------------------------------------
# Build and solve
# --------------------------------------------------------------------------
class AdaptiveOperator:
    pass


def build(t: AdaptiveTree, p: int, coeffs: np.ndarray, f: np.ndarray | None = None) -> AdaptiveOperator:
    """coeffs[leaf, term, point] (leaves in t.leaves order, 3D term order);
    f[leaf, point] optional (folded into the build)."""
    disc = LeafDisc(D3, p)
    pan = Panels(p - 2)
    leaf_rec = {}
    data = {}   # node -> (boundary list, T, h)
    for i, k in enumerate(t.leaves):
        r = t.half_width(k[0])
        lf = leaf_solve(disc, disc.term_ops(r), disc.Q / r, coeffs[i], None if f is None else f[i])
        leaf_rec[k] = lf
        data[k] = (leaf_panels(t, k), lf.T, lf.h)
    merges = {}
    order = sorted(t.internal, key=lambda k: -k[0])   # deepest first
    for k in order:
        kids = children(k)
        node, bdry, Tp, hp = merge_node(pan, [data[c][0] for c in kids], [data[c][1] for c in kids],
                                        [data[c][2] for c in kids])
        merges[k] = node
        data[k] = (bdry, Tp, hp)
        for c in kids:
            del data[c]
    op = AdaptiveOperator()
    op.tree, op.p, op.disc, op.pan = t, p, disc, pan
    op.leaves, op.merges = leaf_rec, merges
    op.root_bdry, op.root_T, op.root_h = data[(0, 0, 0, 0)]
    return op


def root_boundary_points(op: AdaptiveOperator) -> np.ndarray:
    return np.concatenate([panel_points(op.tree, op.pan.q, p_) for _, p_ in op.root_bdry])


def root_D_size(t: AdaptiveTree, p: int) -> int:
    """Size of the root merge's D (the interface points of the top merge)."""
    pan = Panels(p - 2)
    bd = {k: leaf_panels(t, k) for k in t.leaves}
    q2 = pan.q ** 2
    m = 0
    for k in sorted(t.internal, key=lambda k: -k[0]):
        kids = children(k)
        kb = [bd[c] for c in kids]
        m = 0
        for (c1, f1, c2, f2) in INTERFACES[D3]:
            s1 = {(p_[2], p_[3], p_[4]) for f, p_ in kb[c1] if f == f1}
            s2 = {(p_[2], p_[3], p_[4]) for f, p_ in kb[c2] if f == f2}
            a0 = min(x[0] for x in s1)
            b0 = min(x[1] for x in s1)
            size = max(x[0] + x[2] for x in s1) - a0
            m += len(coarse_squares((a0, b0, size), s1, s2)) * q2
        bd[k] = [(f, p_) for f in range(2 * D3) for c in face_children(D3, f) for ff, p_ in kb[c] if ff == f]
    return m


def solve(op: AdaptiveOperator, g_root: np.ndarray, f: np.ndarray | None = None) -> np.ndarray:
    """u at every leaf point, [leaf, point], from root boundary data (root
    boundary order) and, optionally, a source given at solve time (linear
    upward pass of h and g~; without it the build's particular data)."""
    t, disc = op.tree, op.disc
    gts = {k: n.gt for k, n in op.merges.items()}
    vs = {k: lf.v for k, lf in op.leaves.items()}
    if f is not None:
        hs = {}
        for i, k in enumerate(t.leaves):
            lf = op.leaves[k]
            v = np.zeros(disc.p ** 3)
            v[disc.Ii] = sla.lu_solve(lf.lu, f[i][disc.Ii])
            vs[k] = v
            hs[k] = (disc.Q / t.half_width(k[0])) @ v
        for k in sorted(t.internal, key=lambda k: -k[0]):
            node = op.merges[k]
            kids = children(k)
            h_ext = sum(node.Ext[c].T @ hs[ck] for c, ck in enumerate(kids))
            h_int = sum(node.Rint[c] @ hs[ck] for c, ck in enumerate(kids))
            gt = -sla.lu_solve(node.D_lu, h_int)
            gts[k] = gt
            hs[k] = (h_ext + node.B @ gt)[node.perm]
    g = {(0, 0, 0, 0): g_root}
    for k in sorted(t.internal, key=lambda k: k[0]):
        node = op.merges[k]
        ge = np.empty_like(g[k])
        ge[node.perm] = g[k]
        gi = node.S @ ge + gts[k]
        for c, ck in enumerate(children(k)):
            g[ck] = node.Ext[c] @ ge + node.Int[c] @ gi
    u = np.empty((len(t.leaves), disc.p ** 3))
    for i, k in enumerate(t.leaves):
        u[i] = op.leaves[k].Y @ g[k] + vs[k]
    return u
