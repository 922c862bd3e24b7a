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
