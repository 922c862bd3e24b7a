"""The stored 2D leaf factors against the oracle's leaf operator.

Column s of a leaf's factor holds U(0..s, s) in pivot order, then the L
entries of the rows not yet pivoted after step s, in increasing row order
(perm[s] = the row pivoted at step s).  Rebuilding P L_ii = L U from the
downloaded factor and pivot order must give the oracle's L_ii (the interior
block of sum_t diag(c_t) D_t), to rounding; the pivot order must be a
permutation and every multiplier bounded by 1 / (1 - 2^-12) (threshold
partial pivoting on 12-mantissa-bit keys).
"""
import numpy as np
import pytest

from gpu_util import say, var_coeffs
from oracle import hps as ohps

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DEV = "cuda:0"


def _unpack(col_major, perm, ni):
    """(L, U) in pivot order from the compact column layout."""
    C = col_major.reshape(ni, ni).T.copy()  # C[:, s] = stored column s
    pos = np.empty(ni, dtype=np.int64)
    pos[perm] = np.arange(ni)
    Lp = np.eye(ni)
    Up = np.zeros((ni, ni))
    for s in range(ni):
        Up[: s + 1, s] = C[: s + 1, s]
        rows = [r for r in range(ni) if pos[r] > s]          # not yet pivoted, row order
        for t, r in enumerate(rows):
            Lp[pos[r], s] = C[s + 1 + t, s]
    return Lp, Up


@pytest.mark.parametrize("p,L,k", [(6, 2, 0.0), (12, 2, 8.0), (16, 1, 20.0)])
def test_factor_layout_rebuilds_lii(p, L, k):
    import paper_2503_17535_amd as hp
    say(f"[case] factor layout p={p} L={L} k={k}")
    tree = ohps.Tree(2, L)
    disc = ohps.LeafDisc(2, p)
    pts = tree.leaf_points(disc)
    c = var_coeffs(pts, seed=11, k=k)
    op = hp.build(hp.tree(2, L), p, torch.tensor(c, device=DEV))
    ni = (p - 2) ** 2
    nl = tree.n_leaves
    LU = op.download(0)
    perm = op.download(1).astype(np.int64)
    op.free()
    ops = disc.term_ops(tree.leaf_r)
    worst = 0.0
    for leaf in range(nl):
        Lfull = ohps.leaf_operator(disc, ops, c[leaf])
        Lii = Lfull[np.ix_(disc.Ii, disc.Ii)]
        pl = perm[leaf * ni:(leaf + 1) * ni]
        assert sorted(pl.tolist()) == list(range(ni))
        Lp, Up = _unpack(LU[leaf * ni * ni:(leaf + 1) * ni * ni], pl, ni)
        assert np.max(np.abs(np.tril(Lp, -1))) <= 1.0 / (1.0 - 2.0 ** -12)
        err = np.max(np.abs(Lp @ Up - Lii[pl])) / np.max(np.abs(Lii))
        worst = max(worst, err)
    say(f"[case] max |P L_ii - L U| / max |L_ii| = {worst:.2e}")
    assert worst < 1e-13
