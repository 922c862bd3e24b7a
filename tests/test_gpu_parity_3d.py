"""3D GPU parity against the oracle: uniform octrees with the div(a grad u)
operator of the 3D workload (a = 1 + 0.5 sin-product, first-order terms grad a)
and with every coefficient term on.  Leaves of n_i = (p-2)^3 unknowns are
inverted by the register Gauss-Jordan (n_i <= 224) or the blocked one."""
import numpy as np
import pytest

import workloads as W
from gpu_util import oracle_solve, rel_inf, rhs, say, var_coeffs
from oracle import hps as ohps

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
TOL = 1e-10


def _run3d(p, L, nrhs, kind="divgrad", with_src=True):
    import paper_2503_17535_amd as hp
    say(f"[case] 3D p={p} L={L} nrhs={nrhs} kind={kind}")
    tree = ohps.Tree(3, L)
    disc = ohps.LeafDisc(3, p)
    pts = tree.leaf_points(disc)
    bpts = tree.root_boundary_points(disc)
    if kind == "divgrad":
        c = W.coeffs_divgrad(pts, W.draw_sinprod(W.rng(3, 0)))
    else:
        c = var_coeffs(pts, 1, 0.0, True)
    bd, src = rhs(pts, bpts, nrhs, 5)
    if not with_src:
        src = None
    ref = oracle_solve(3, p, L, c, bd, src)
    dev = torch.device("cuda:0")
    op = hp.build(hp.tree(3, L), p, torch.tensor(c, device=dev))
    u = op.solve(torch.tensor(bd, device=dev), None if src is None else torch.tensor(src, device=dev))
    err = rel_inf(u.cpu().numpy(), ref)
    op.free()
    say(f"[case] rel err {err:.3e}")
    return err


@pytest.mark.parametrize("p,L", [(6, 1), (8, 1), (6, 2), (12, 1)])
def test_parity_3d_divgrad(p, L):
    assert _run3d(p, L, 2) < TOL


def test_parity_3d_all_terms():
    assert _run3d(5, 2, 3, kind="all") < TOL


def test_parity_3d_no_source():
    assert _run3d(7, 1, 1, with_src=False) < TOL


def test_3d_manufactured_solution_accuracy():
    """div(a grad u) = f with u = sin(pi x) sin(pi y) sin(pi z) + xyz (the 3D
    workload's data): the GPU solution converges to the exact u."""
    import paper_2503_17535_amd as hp
    say("[case] 3D manufactured p=10 L=1")
    p, L = 10, 1
    t = hp.tree(3, L)
    pts = hp.leaf_points(t, p)
    bpts = hp.boundary_points(t, p)
    prm = W.draw_sinprod(W.rng(3, 0))
    c = W.coeffs_divgrad(pts, prm)
    f = W.divgrad_source(prm, pts)
    g = W.sin3_plus_xyz(bpts)[0]
    dev = torch.device("cuda:0")
    op = hp.build(t, p, torch.tensor(c, device=dev))
    u = op.solve(torch.tensor(g[None], device=dev), torch.tensor(f[None], device=dev)).cpu().numpy()[0]
    op.free()
    ue = W.sin3_plus_xyz(pts)[0]
    err = np.abs(u - ue).max() / np.abs(ue).max()
    say(f"[case] error vs exact {err:.3e}")
    assert err < 1e-3


def _poly3(pts, deg):
    """u = prod_a P_a(x_a) with per-variable degree `deg`, its gradient and
    Laplacian (closed form)."""
    from numpy.polynomial import polynomial as npoly
    coefs = [np.array([0.2, -0.3, 0.1, 0.05] + [0.0] * (deg - 4) + [0.4 + 0.1 * a]) for a in range(3)]
    vals = [npoly.polyval(pts[..., a], coefs[a]) for a in range(3)]
    d1 = [npoly.polyval(pts[..., a], npoly.polyder(coefs[a])) for a in range(3)]
    d2 = [npoly.polyval(pts[..., a], npoly.polyder(coefs[a], 2)) for a in range(3)]
    u = vals[0] * vals[1] * vals[2]
    grad = np.stack([d1[0] * vals[1] * vals[2], vals[0] * d1[1] * vals[2], vals[0] * vals[1] * d1[2]], axis=-1)
    lap = d2[0] * vals[1] * vals[2] + vals[0] * d2[1] * vals[2] + vals[0] * vals[1] * d2[2]
    return u, grad, lap


def _divgrad_full(kind):
    # the 3D workload at full size: div(a grad u) = f on [-1,1]^3, a = 1 + 0.5
    # sin-product, depth 3 (512 leaves), p = 12; root D = 19,200 (block inversion)
    import paper_2503_17535_amd as hp
    p, L = 12, 3
    t = hp.tree(3, L)
    pts = hp.leaf_points(t, p)
    bpts = hp.boundary_points(t, p)
    prm = W.draw_sinprod(W.rng(3, 0))
    c = W.coeffs_divgrad(pts, prm)
    a, ga = W.eval_sinprod(prm, pts)
    if kind == "poly":
        ue, gu, lap = _poly3(pts, p - 3)
        g = _poly3(bpts, p - 3)[0]
    else:
        ue, gu, lap = W.sin3_plus_xyz(pts)
        g = W.sin3_plus_xyz(bpts)[0]
    f = a * lap + np.sum(ga * gu, axis=-1)
    dev = torch.device("cuda:0")
    op = hp.build(t, p, torch.tensor(c, device=dev))
    say(f"[case] built: {op.nbytes / 1e9:.2f} GB resident")
    u = op.solve(torch.tensor(g[None], device=dev), torch.tensor(f[None], device=dev)).cpu().numpy()[0]
    op.free()
    return np.abs(u - ue).max() / np.abs(ue).max()


def test_3d_full_size_polynomial_exactness():
    """For u polynomial of per-variable degree p-3 every interpolation and
    differentiation of the discretization is exact, so the discrete solution
    is u up to rounding at any size (here the 3D workload's full size)."""
    say("[case] 3D full size p=12 L=3, polynomial u")
    err = _divgrad_full("poly")
    say(f"[case] rel error vs exact polynomial {err:.3e}")
    assert err < 1e-10


def test_3d_full_size_manufactured_solution():
    say("[case] 3D full size p=12 L=3, u = sin sin sin + xyz")
    err = _divgrad_full("sin")
    say(f"[case] rel error vs exact {err:.3e}")
    assert err < 1e-5
