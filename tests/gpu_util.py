"""Shared helpers of the GPU tests: seeded inputs on the oracle's points and
the oracle's solution for them."""
import sys

import numpy as np

import workloads as W
from oracle import hps as ohps


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def var_coeffs(pts, seed=0, k=0.0, mixed=True):
    """Smooth variable coefficients (every term on), optionally Helmholtz-like."""
    d = pts.shape[-1]
    g = np.random.default_rng(seed)
    a1, a2, a3 = g.uniform(0.5, 1.5, 3)
    x, y = pts[..., 0], pts[..., 1]
    c = W.coeffs_poisson(pts)
    c[:, 0, :] = -(1.0 + 0.2 * np.sin(a1 * x + 2 * y))
    if d == 2:
        if mixed:
            c[:, 1, :] = 0.1 * np.cos(a2 * x * y)
        c[:, 2, :] = -(1.0 + 0.2 * np.cos(x - a3 * y))
        c[:, 3, :] = 0.3 * np.cos(3 * y)
        c[:, 4, :] = -0.2 * np.sin(2 * x)
    else:
        c[:, 6, :] = 0.3 * np.cos(3 * y)
        c[:, 8, :] = 0.2 * x
        if mixed:
            c[:, 3, :] = 0.1 * np.cos(x)
    c[:, -1, :] = -(k * k) * (1.0 + 0.3 * np.sin(3 * x) * np.cos(y)) - 0.5
    return c


def rhs(pts, bpts, nrhs, seed=0):
    g = np.random.default_rng(1000 + seed)
    bd = np.empty((nrhs, bpts.shape[0]))
    src = np.empty((nrhs,) + pts.shape[:-1])
    for r in range(nrhs):
        w = g.uniform(-2, 2, size=(3, pts.shape[-1]))
        bd[r] = np.cos(bpts @ w[0]) + np.sin(bpts @ w[1])
        src[r] = np.exp(-np.sum((pts - 0.3 * w[2]) ** 2, axis=-1) * 4.0) * g.normal()
    return bd, src


def oracle_solve(d, p, L, coeffs, bd, src):
    tree = ohps.Tree(d, L)
    op = ohps.build(tree, p, coeffs)
    out = []
    for r in range(bd.shape[0]):
        out.append(ohps.solve(op, bd[r], None if src is None else src[r]))
    return np.stack(out)


def rel_inf(u, ref):
    """max over right-hand sides of ||u - ref||_inf / ||ref||_inf"""
    return max(np.abs(u[r] - ref[r]).max() / np.abs(ref[r]).max() for r in range(ref.shape[0]))


def composite_solve(tree, p, coeffs, bd_r, bpts, src_r):
    """Solution of the composite collocation system (oracle.dense, sparse LU)
    for boundary values bd_r given at the root boundary points bpts.  In exact
    arithmetic it equals the HPS solution, so its distance to the HPS oracle
    measures how far rounding alone moves the result for this problem."""
    import scipy.sparse.linalg as spla
    from oracle import dense

    def g_fun(x):
        d2 = ((x[:, None, :] - bpts[None, :, :]) ** 2).sum(-1)
        j = d2.argmin(axis=1)
        assert np.all(d2[np.arange(len(j)), j] < 1e-24)
        return bd_r[j]

    K, layout = dense.assemble(tree, p, coeffs, sparse=True)
    b = dense.rhs(tree, layout, src_r, g_fun)
    x = spla.splu(K.tocsc()).solve(b)
    return x[:layout["n_u"]].reshape(tree.n_leaves, p ** tree.d)


def rounding_spread(tree, p, coeffs, bd, bpts, src, ref):
    """max over rhs of the relative distance between the HPS oracle (ref) and
    the composite-system solution: the spread of two fp64 computations of the
    same exact result."""
    alt = np.stack([composite_solve(tree, p, coeffs, bd[r], bpts, None if src is None else src[r])
                    for r in range(bd.shape[0])])
    return rel_inf(alt, ref)


def merge_conditioning(tree, p, coeffs):
    """cond_2(D) of every merge matrix of the oracle's tree, as
    {m: (max, median)} (the conditioning the merges' inverses work under)."""
    from oracle import hps as H
    disc = ohps.LeafDisc(tree.d, p)
    ops = disc.term_ops(tree.leaf_r)
    Qr = disc.Q / tree.leaf_r
    T = []
    h = []
    for i in range(tree.n_leaves):
        lf = ohps.leaf_solve(disc, ops, Qr, coeffs[i], None)
        T.append(lf.T)
        h.append(lf.h)
    nd = 2 ** tree.d
    n = disc.n_face
    out = {}
    for lev in range(tree.L - 1, -1, -1):
        Tn, hn, cs = [], [], []
        for j in range(len(T) // nd):
            kids = slice(nd * j, nd * j + nd)
            if tree.d == 2:
                D = H.merge_blocks_2d(T[kids], h[kids], n)[3]
            else:
                D = H.merge_blocks_general(tree.d, T[kids], h[kids], n)[3]
            cs.append(np.linalg.cond(D))
            if lev > 0:
                _, Tp, hp = H.merge(tree.d, T[kids], h[kids], n)
                Tn.append(Tp)
                hn.append(hp)
        out[D.shape[0]] = (float(max(cs)), float(np.median(cs)))
        T, h = Tn, hn
        n *= 2 ** (tree.d - 1)
    return out


def cond_by_level(op_o):
    """cond_1(D) of the oracle operator's merges, per tree level (root
    first) as (m, max, median): the conditioning every parity number of a
    Helmholtz workload is reported with."""
    out = []
    for nodes in op_o.levels:
        cs = [nd.cond1 for nd in nodes]
        m = nodes[0].S.shape[0]
        out.append((m, float(np.max(cs)), float(np.median(cs))))
    return out


def fmt_cond(conds):
    return ", ".join(f"m={m}: {mx:.1e}/{md:.1e}" for m, mx, md in conds)
