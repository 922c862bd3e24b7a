"""One-dimensional spectral building blocks of the HPS discretization (fp64).

Test infrastructure only (see the package docstring).

* Chebyshev--Lobatto nodes, ascending: x_j = -cos(pi j / (p-1))  (Section 3.1:
  a tensor product of order-p Chebyshev--Lobatto points per leaf).
* Gauss--Legendre nodes and weights of order q = p - 2 on each leaf side
  (Section 3.1), computed here by the Golub--Welsch eigenvalue method.
* Barycentric Lagrange interpolation and the spectral differentiation matrix
  (Section 3.2 and Appendix A.1: differentiation matrices in the style of
  Trefethen, and barycentric interpolation between Chebyshev and Gauss points).

Every routine is the plain textbook definition: barycentric weights by their
product formula, the differentiation matrix from those weights, interpolation
by the second barycentric formula.
"""
from __future__ import annotations

import numpy as np


def cheb_lobatto(p: int) -> np.ndarray:
    """p Chebyshev--Lobatto points on [-1, 1], ascending."""
    j = np.arange(p)
    x = -np.cos(np.pi * j / (p - 1))
    if p % 2 == 1:
        x[p // 2] = 0.0
    return x


def gauss_legendre(q: int):
    """Golub--Welsch: nodes are the eigenvalues of the symmetric Jacobi matrix
    of the Legendre recurrence (off-diagonal k / sqrt(4k^2 - 1)); weights are
    2 * (first eigenvector component)^2.  Returned ascending."""
    k = np.arange(1, q)
    off = k / np.sqrt(4.0 * k * k - 1.0)
    J = np.diag(off, 1) + np.diag(off, -1)
    lam, V = np.linalg.eigh(J)
    w = 2.0 * V[0, :] ** 2
    order = np.argsort(lam)
    return lam[order], w[order]


def bary_weights(x: np.ndarray) -> np.ndarray:
    """w_j = 1 / prod_{k != j} (x_j - x_k)."""
    n = len(x)
    w = np.empty(n)
    for j in range(n):
        d = x[j] - np.delete(x, j)
        w[j] = 1.0 / np.prod(d)
    return w


def diff_matrix(x: np.ndarray) -> np.ndarray:
    """Spectral differentiation matrix of the polynomial interpolant through
    nodes x: D_ij = (w_j / w_i) / (x_i - x_j) for i != j and
    D_ii = -sum_{j != i} D_ij."""
    n = len(x)
    w = bary_weights(x)
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = (w[j] / w[i]) / (x[i] - x[j])
        D[i, i] = -np.sum(D[i, :])
    return D


def interp_matrix(x_from: np.ndarray, y_to: np.ndarray) -> np.ndarray:
    """Matrix M with (M f)(y_i) = interpolant of (x_from, f) at y_i, by the
    second (true) barycentric formula; exact node hits copy the value."""
    w = bary_weights(x_from)
    M = np.zeros((len(y_to), len(x_from)))
    for i, y in enumerate(y_to):
        diff = y - x_from
        hit = np.nonzero(np.abs(diff) < 1e-15)[0]
        if hit.size:
            M[i, hit[0]] = 1.0
            continue
        t = w / diff
        M[i, :] = t / np.sum(t)
    return M
