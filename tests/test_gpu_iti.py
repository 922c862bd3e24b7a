"""GPU parity of the ItI variant (Appendix B; hps_build_iti) against the CPU
oracle ``oracle.iti`` on the same seeded inputs: complex incoming impedance
data at the root Gauss points, complex sources, real variable coefficients
(Helmholtz-like).  Bar: rel. l_inf <= 1e-10 per right-hand side (the solver's
fp64 bar).  Sizes span one leaf level to four merge levels, the blocked and
single-workgroup Gauss-Jordan forms (B is 2p^2 reals per leaf: 72 at p = 6,
128 at p = 8, 288 at p = 12, 512 at p = 16), source-free solves and the
16-rhs chunking; at p = 16, depth 5 the solve reproduces a polynomial
solution (property that holds at any size), and the paper's ItI problem is
checked against its exact solution.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import say, var_coeffs
from oracle import hps as H
from oracle import iti as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DEV = "cuda:0"
TOL = 1e-10


def _data(pts, bpts, nrhs, seed):
    g = np.random.default_rng(2000 + seed)
    bd = np.empty((nrhs, bpts.shape[0]), dtype=complex)
    src = np.empty((nrhs,) + pts.shape[:-1], dtype=complex)
    for r in range(nrhs):
        w = g.uniform(-2, 2, size=(4, 2))
        bd[r] = np.cos(bpts @ w[0]) + 1j * np.sin(bpts @ w[1])
        amp = g.normal() + 1j * g.normal()
        src[r] = amp * np.exp(-np.sum((pts - 0.3 * w[2]) ** 2, axis=-1) * 4.0)
    return bd, src


def _rel(u, ref):
    return max(np.abs(u[r] - ref[r]).max() / np.abs(ref[r]).max() for r in range(ref.shape[0]))


def _run(p, L, nrhs, eta=2.0, k=3.0, seed=0, with_src=True):
    import paper_2503_17535_amd as hp
    say(f"[case] ItI p={p} L={L} nrhs={nrhs} eta={eta} k={k} src={with_src}")
    tree = H.Tree(2, L)
    disc = H.LeafDisc(2, p)
    pts = tree.leaf_points(disc)
    bpts = tree.root_boundary_points(disc)
    c = var_coeffs(pts, seed, k, mixed=True)
    bd, src = _data(pts, bpts, nrhs, seed)
    if not with_src:
        src = None
    op_o = I.build(tree, p, eta, c)
    ref = np.stack([I.solve(op_o, bd[r], None if src is None else src[r]) for r in range(nrhs)])
    op = hp.build_iti(hp.tree(2, L), p, torch.tensor(c, device=DEV), eta)
    u = op.solve(torch.tensor(bd, device=DEV), None if src is None else torch.tensor(src, device=DEV))
    torch.cuda.synchronize()
    err = _rel(u.cpu().numpy(), ref)
    say(f"[case] rel err {err:.3e}")
    op.free()
    return err


@pytest.mark.parametrize("p,L,nrhs", [(8, 1, 2), (8, 2, 1), (6, 3, 3), (12, 2, 2), (10, 3, 1)])
def test_iti_parity_small(p, L, nrhs):
    assert _run(p, L, nrhs) < TOL


def test_iti_parity_no_source_and_chunks():
    assert _run(6, 2, 18, with_src=False) < TOL


def test_iti_parity_p16_wavenumber():
    # k = 12 on a depth-2 tree: the DtN sub-rectangle problems pass near
    # resonances at such k; the ItI merges stay well posed
    assert _run(16, 2, 2, eta=12.0, k=12.0) < TOL


def _robin_poly(bpts, eta):
    u, d = W.poly5(bpts)
    ux, uy = d[3], d[4]
    x, y = bpts[:, 0], bpts[:, 1]
    un = np.where(np.isclose(y, -1.0), -uy, np.where(np.isclose(x, 1.0), ux, np.where(np.isclose(y, 1.0), uy, -ux)))
    return un + 1j * eta * u


def test_iti_polynomial_depth5_p16():
    """A degree-5 polynomial with variable coefficients: reproduced to
    rounding at 1024 leaves (bar 1e-13 4^depth, as for the DtN variant)."""
    import paper_2503_17535_amd as hp
    L, p, eta = 5, 16, 4.0
    say(f"[case] ItI polynomial depth {L} p {p}")
    t = hp.tree(2, L)
    pts = hp.leaf_points(t, p)
    bpts = hp.boundary_points(t, p)
    c, f, _, uex = W.poly5_problem(pts, bpts)
    g = _robin_poly(bpts, eta)
    op = hp.build_iti(t, p, torch.tensor(c, device=DEV), eta)
    u = op.solve(torch.tensor(g[None], device=DEV), torch.tensor(f[None].astype(complex), device=DEV))
    torch.cuda.synchronize()
    err = np.abs(u[0].cpu().numpy() - uex).max() / np.abs(uex).max()
    say(f"[case] rel err vs exact polynomial {err:.3e}")
    op.free()
    assert err < 1e-13 * 4.0 ** L


def test_iti_paper_problem():
    """The paper's ItI problem (eq. ItI_problem, eta = 1), p = 12, depth 3:
    GPU against the oracle (1e-10) and both against the exact solution."""
    import paper_2503_17535_amd as hp
    p, L = 12, 3
    say(f"[case] ItI paper problem p={p} L={L}")
    tree = H.Tree(2, L)
    disc = H.LeafDisc(2, p)
    pts = tree.leaf_points(disc)
    bpts = tree.root_boundary_points(disc)
    x, y = pts[..., 0], pts[..., 1]
    c = np.zeros((tree.n_leaves, 6, p * p))
    c[:, 0] = 1.0
    c[:, 2] = 1.0
    c[:, 5] = 1.0 + np.exp(-50 * (x ** 2 + y ** 2))
    uex = np.exp(20j * x) + np.exp(30j * y)
    f = -400 * np.exp(20j * x) - 900 * np.exp(30j * y) + c[:, 5] * uex
    bx, by = bpts[:, 0], bpts[:, 1]
    ub = np.exp(20j * bx) + np.exp(30j * by)
    ux, uy = 20j * np.exp(20j * bx), 30j * np.exp(30j * by)
    un = np.where(np.isclose(by, -1), -uy, np.where(np.isclose(bx, 1), ux, np.where(np.isclose(by, 1), uy, -ux)))
    g = un + 1j * ub
    ref = I.solve(I.build(tree, p, 1.0, c), g, f)
    op = hp.build_iti(hp.tree(2, L), p, torch.tensor(c, device=DEV), 1.0)
    u = op.solve(torch.tensor(g[None], device=DEV), torch.tensor(f[None], device=DEV))[0].cpu().numpy()
    op.free()
    ii = disc.Ii
    e_gpu = np.abs(u[:, ii] - uex[:, ii]).max() / np.abs(uex[:, ii]).max()
    e_ora = np.abs(ref[:, ii] - uex[:, ii]).max() / np.abs(uex[:, ii]).max()
    par = np.abs(u - ref).max() / np.abs(ref).max()
    say(f"[case] vs oracle {par:.3e}; vs exact: GPU {e_gpu:.3e}, oracle {e_ora:.3e}")
    assert par < TOL
    assert abs(e_gpu - e_ora) <= 1e-9


def test_iti_rejects_other_calls():
    import paper_2503_17535_amd as hp
    say("[case] ItI: unsupported calls")
    t = hp.tree(2, 2)
    s = hp.sizes(t, 8)
    c = torch.tensor(var_coeffs(hp.leaf_points(t, 8)), device=DEV)
    op = hp.build_iti(t, 8, c, 1.0)
    w = torch.zeros((1, s.n_leaves, s.pts_per_leaf), dtype=torch.float64, device=DEV)
    with pytest.raises(hp.HPSError) as e:
        hp.Operator.solve_adjoint(op, w)
    assert e.value.code == hp.HPS_EUNSUPPORTED
    with pytest.raises(hp.HPSError) as e:
        op.level_info()
    assert e.value.code == hp.HPS_EUNSUPPORTED
    op.free()
