"""CPU check of the block elimination the library uses for large merge
matrices (Algorithm merge, "Invert D"), on the oracle's own D matrices.

D's interfaces split as [P1 | P2 | R] with D(P1, P2) = D(P2, P1) = 0
(2D: interfaces 5 = a|b and 7 = c|d share no child).  The inverse follows from
the inverses of D(P_b, P_b), the Schur complement
Sc = D(R,R) - sum_b D(R,P_b) D(P_b,P_b)^{-1} D(P_b,R) and its inverse.  That
pivots only inside the blocks.  These tests show, with numpy's partially
pivoted inverses standing in for the blocks:
* at the root merge of the smoke workload (Helmholtz k = 10, p = 12, depth 3)
  the blocks are ill conditioned and the block inverse misses by > 1e-9
  while a pivoted inverse of all of D is at rounding level: the guard's probe
  |Z (D x) - x| / |x| trips;
* one Newton-Schulz step Z <- 2Z - Z (D Z) restores rounding level, and two
  steps suffice over a sweep of wavenumbers near sub-rectangle resonances."""
import numpy as np
import pytest

import workloads as W
from oracle import hps as ohps


def _merge_matrices(k, p, L):
    """D of every merge of the oracle's build (levels root first), formed
    with the oracle's own leaf solves and Appendix A.2 blocks."""
    tree = ohps.Tree(2, L)
    disc = ohps.LeafDisc(2, p)
    pts = tree.leaf_points(disc)
    c, _, _ = W.helmholtz_inputs(pts, tree.root_boundary_points(disc), k, 1)
    ops = disc.term_ops(tree.leaf_r)
    Qr = disc.Q / tree.leaf_r
    leaves = [ohps.leaf_solve(disc, ops, Qr, c[i]) for i in range(tree.n_leaves)]
    T, h = [lf.T for lf in leaves], [lf.h for lf in leaves]
    n, levels = disc.n_face, []
    for lev in range(L - 1, -1, -1):
        Ds, Tn, hn = [], [], []
        for j in range(len(T) // 4):
            kids = slice(4 * j, 4 * j + 4)
            Ds.append(ohps.merge_blocks_2d(T[kids], h[kids], n)[3])
            _, Tp, hp = ohps.merge(2, T[kids], h[kids], n, with_T=lev > 0)
            Tn.append(Tp)
            hn.append(hp)
        levels.append(Ds)
        T, h = Tn, hn
        n *= 2
    return levels[::-1]


def _block_inverse(D):
    m = D.shape[0]
    n = m // 4
    order = np.r_[np.arange(0, n), np.arange(2 * n, 3 * n), np.arange(n, 2 * n), np.arange(3 * n, 4 * n)]
    Dp = D[np.ix_(order, order)]
    s = n
    assert np.all(Dp[:s, s:2 * s] == 0) and np.all(Dp[s:2 * s, :s] == 0)
    Ai = [np.linalg.inv(Dp[b * s:(b + 1) * s, b * s:(b + 1) * s]) for b in range(2)]
    X = [Ai[b] @ Dp[b * s:(b + 1) * s, 2 * s:] for b in range(2)]
    Y = [Dp[2 * s:, b * s:(b + 1) * s] @ Ai[b] for b in range(2)]
    Sc = Dp[2 * s:, 2 * s:] - sum(Dp[2 * s:, b * s:(b + 1) * s] @ X[b] for b in range(2))
    Sci = np.linalg.inv(Sc)
    Z = np.zeros_like(Dp)
    Z[2 * s:, 2 * s:] = Sci
    for b in range(2):
        Z[b * s:(b + 1) * s, 2 * s:] = -X[b] @ Sci
        Z[2 * s:, b * s:(b + 1) * s] = -Sci @ Y[b]
    for b in range(2):
        for cc in range(2):
            Z[b * s:(b + 1) * s, cc * s:(cc + 1) * s] = (Ai[b] if b == cc else 0) - Z[b * s:(b + 1) * s, 2 * s:] @ Y[cc]
    inv = np.empty(m, dtype=int)
    inv[order] = np.arange(m)
    return Z[np.ix_(inv, inv)]


def _probe(D, Z):
    # the right residual D (Z x) - x on four pseudo-random vectors, as the
    # library probes its block-eliminated inverses
    x = np.random.default_rng(7).uniform(-1, 1, size=(D.shape[0], 4))
    return np.abs(D @ (Z @ x) - x).max() / np.abs(x).max()


def _newton_schulz(D, Z):
    return 2 * Z - Z @ (D @ Z)


def test_block_inverse_trips_guard_at_smoke_root():
    Droot = _merge_matrices(10.0, 12, 3)[0][0]
    assert Droot.shape == (160, 160)
    Zb = _block_inverse(Droot)
    Zp = np.linalg.inv(Droot)
    assert _probe(Droot, Zp) < 1e-13
    assert _probe(Droot, Zb) > 1e-9          # the loss the guard must catch
    assert _probe(Droot, _newton_schulz(Droot, Zb)) < 1e-13
    # the refined inverse equals the pivoted one to rounding
    Z1 = _newton_schulz(Droot, Zb)
    assert np.abs(Z1 - Zp).max() < 1e-12 * np.abs(Zp).max()


@pytest.mark.parametrize("k", [9.0, 9.93, 12.0, 14.05, 20.0])
def test_two_steps_suffice_near_resonances(k):
    # refined as the library does (a step while the probe is above 1e-12, at
    # most two), the block inverse is as accurate as a pivoted inverse of all
    # of D (whose own residual grows with cond(D): 1e-12 at cond 3.5e4)
    for nodes in _merge_matrices(k, 12, 3):
        for D in nodes:
            Z = _block_inverse(D)
            for _ in range(2):
                if _probe(D, Z) <= 1e-12:
                    break
                Z = _newton_schulz(D, Z)
            floor = _probe(D, np.linalg.inv(D))
            assert _probe(D, Z) < max(1e-12, 10 * floor), (k, D.shape)
            assert _probe(D, Z) < 1e-10
