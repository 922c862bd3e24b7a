"""GPU parity of the adjoint solve, the coefficient gradient and the
torch.autograd binding against the CPU oracle, plus properties that hold at
any size (the dot-product identity) and central finite differences.

Tolerances: lam_src and lam_bdry are solutions of the transposed system, so
they carry the fp64 solve bar (rel. l_inf <= 1e-10).  The gradient is the
product k^2 u lam of two such fields: |d(u lam)| <= (e_u + e_lam) max|u|
max|lam|, i.e. 2e-10 of that scale."""
import numpy as np
import pytest

import workloads as W
from gpu_util import rhs, say, var_coeffs
from oracle import adjoint as A
from oracle import hps as ohps

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-10
DEV = "cuda:0"


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("d,p,L,nrhs,k", [(2, 8, 2, 3, 0.0), (2, 16, 3, 2, 10.0), (2, 7, 4, 20, 2.0),
                                          (3, 6, 1, 2, 0.0), (3, 5, 2, 1, 1.0)])
def test_adjoint_matches_oracle(d, p, L, nrhs, k):
    import paper_2503_17535_amd as hp
    say(f"[case] adjoint d={d} p={p} L={L} nrhs={nrhs} k={k}")
    tree = ohps.Tree(d, L)
    disc = ohps.LeafDisc(d, p)
    pts = tree.leaf_points(disc)
    c = var_coeffs(pts, seed=3, k=k)
    w = np.random.default_rng(21).normal(size=(nrhs,) + pts.shape[:-1])
    op_o = ohps.build(tree, p, c)
    ref = [A.hps_adjoint(op_o, w[r]) for r in range(nrhs)]
    t = hp.tree(d, L)
    op = hp.build(t, p, torch.tensor(c, device=DEV))
    lb = torch.empty((nrhs, op.sizes.n_root_bdry), dtype=torch.float64, device=DEV)
    ls, lb = op.solve_adjoint(torch.tensor(w, device=DEV), lam_bdry=lb)
    ls, lb = ls.cpu().numpy(), lb.cpu().numpy()
    op.free()
    es = max(_rel(ls[r], ref[r][0]) for r in range(nrhs))
    eb = max(_rel(lb[r], ref[r][1]) for r in range(nrhs))
    say(f"[case] lam_src rel err {es:.3e}  lam_bdry rel err {eb:.3e}")
    assert es < TOL and eb < TOL
    assert np.all(ls[:, :, disc.Ie] == 0.0)


def test_adjoint_dot_product_full_size():
    # 2D Helmholtz k = 40, depth 6 (4096 leaves), p = 16, 16 right-hand sides
    import paper_2503_17535_amd as hp
    say("[case] adjoint dot product, Helmholtz k=40 L=6 p=16, 16 rhs")
    d, p, L, nrhs = 2, 16, 6, 16
    t = hp.tree(d, L)
    pts = hp.leaf_points(t, p)
    bpts = hp.boundary_points(t, p)
    c, bd, src = W.helmholtz_inputs(pts, bpts, 40.0, nrhs)
    op = hp.build(t, p, torch.tensor(c, device=DEV))
    bd_t, src_t = torch.tensor(bd, device=DEV), torch.tensor(src, device=DEV)
    u = op.solve(bd_t, src_t)
    w = torch.randn(u.shape, dtype=torch.float64, device=DEV, generator=torch.Generator(DEV).manual_seed(5))
    lb = torch.empty_like(bd_t)
    ls, lb = op.solve_adjoint(w, lam_bdry=lb)
    lhs = (w * u).sum(dim=(1, 2))
    rhs_ = (ls * src_t).sum(dim=(1, 2)) + (lb * bd_t).sum(dim=1)
    scale = w.norm(dim=(1, 2)) * u.norm(dim=(1, 2))
    err = ((lhs - rhs_).abs() / scale).max().item()
    op.free()
    say(f"[case] dot-product identity rel err {err:.3e}")
    assert err < 1e-12


@pytest.mark.parametrize("d,p,L", [(2, 10, 2), (3, 6, 1)])
def test_coeff_grad_matches_oracle(d, p, L):
    import paper_2503_17535_amd as hp
    say(f"[case] coeff grad d={d} p={p} L={L}")
    tree = ohps.Tree(d, L)
    disc = ohps.LeafDisc(d, p)
    pts = tree.leaf_points(disc)
    bpts = tree.root_boundary_points(disc)
    c = var_coeffs(pts, seed=4, k=1.0)
    bd, src = rhs(pts, bpts, 2, seed=4)
    w = np.random.default_rng(22).normal(size=(2,) + pts.shape[:-1])
    op_o = ohps.build(tree, p, c)
    u_o = np.stack([ohps.solve(op_o, bd[r], src[r]) for r in range(2)])
    l_o = np.stack([A.hps_adjoint(op_o, w[r])[0] for r in range(2)])
    ref = A.coeff_grad(tree, p, u_o, l_o)
    op = hp.build(hp.tree(d, L), p, torch.tensor(c, device=DEV))
    u = op.solve(torch.tensor(bd, device=DEV), torch.tensor(src, device=DEV))
    lam, _ = op.solve_adjoint(torch.tensor(w, device=DEV))
    g = op.coeff_grad(u, lam).cpu().numpy()
    op.free()
    errs = [_rel(g[:, t], ref[:, t]) for t in range(c.shape[1])]
    say("[case] coeff grad rel err per term " + " ".join(f"{e:.2e}" for e in errs))
    # d_t u of a field with relative error e has error up to |D_t| e max|u|:
    # allow 10x the solve bar per term
    assert max(errs) < 10 * TOL
    assert np.all(g[:, :, disc.Ie] == 0.0)


def _helmholtz_coeffs(q, k):
    """Differentiable coefficients of -Lap u - k^2 (1 + q) u from q [nl, np]."""
    nl, npts = q.shape
    c = torch.zeros((nl, 6, npts), dtype=torch.float64, device=q.device)
    c[:, 0] = -1.0
    c[:, 2] = -1.0
    return torch.cat([c[:, :5], (-(k * k) * (1.0 + q))[:, None]], dim=1)


def test_autograd_misfit_gradient_differentiation_workload():
    # misfit at 256 points, 2D Helmholtz k = 20, depth 5, p = 16, 32 fields
    import paper_2503_17535_amd as hp
    from paper_2503_17535_amd.autograd import solve as hsolve
    d, p, L = 2, 16, 5
    say("[case] autograd misfit gradient, k=20 L=5 p=16, 32 fields")
    t = hp.tree(d, L)
    pts = hp.leaf_points(t, p)
    bpts = hp.boundary_points(t, p)
    inp = W.differentiation_inputs(pts, bpts)
    k = inp["k"]
    bd = torch.tensor(inp["bdry"], device=DEV)
    src = torch.tensor(inp["src"], device=DEV)
    leaf, wts = hp.interp_weights(t, p, inp["x_obs"])
    leaf_t, wts_t = torch.tensor(leaf, device=DEV), torch.tensor(wts, device=DEV)

    def observe(u):
        return (wts_t * u[0, leaf_t, :]).sum(-1)

    with torch.no_grad():
        u_star = hsolve(t, p, _helmholtz_coeffs(torch.tensor(inp["q_star"], device=DEV), k), bd, src)
        u_obs = observe(u_star)

    def J_of(qt):
        u = hsolve(t, p, _helmholtz_coeffs(qt, k), bd, src)
        return ((observe(u) - u_obs) ** 2).sum(), u

    grads = []
    for f in range(inp["q"].shape[0]):
        q = torch.tensor(inp["q"][f], device=DEV, requires_grad=True)
        J, _ = J_of(q)
        J.backward()
        grads.append(q.grad.detach())
        assert torch.isfinite(q.grad).all() and q.grad.abs().max() > 0
    say("[case] 32 gradients done")
    g0 = grads[0].cpu().numpy()

    # oracle gradient of field 0: its own solves, observation operator and adjoint
    tree = ohps.Tree(d, L)
    disc = ohps.LeafDisc(d, p)
    opts = tree.leaf_points(disc)
    c_star = W.coeffs_helmholtz(opts, k, inp["q_star"])
    op_s = ohps.build(tree, p, c_star)
    oleaf, oW = A.observation(tree, p, inp["x_obs"])
    uo_obs = np.einsum("mk,mk->m", oW, ohps.solve(op_s, inp["bdry"][0], inp["src"][0])[oleaf])
    del op_s
    op0 = ohps.build(tree, p, W.coeffs_helmholtz(opts, k, inp["q"][0]))
    u0 = ohps.solve(op0, inp["bdry"][0], inp["src"][0])
    lam0, _ = A.hps_adjoint(op0, A.misfit_weight(u0, oleaf, oW, uo_obs))
    ref = -(k * k) * A.coeff_grad(tree, p, u0[None], lam0[None])[:, 5]
    scale = k * k * np.abs(u0).max() * np.abs(lam0).max()
    err = np.abs(g0 - ref).max()
    say(f"[case] oracle gradient abs err {err:.3e}, scale {scale:.3e}, rel {err / np.abs(ref).max():.3e}")
    assert err < 2 * TOL * scale
    assert np.all(g0[:, disc.Ie] == 0.0)

    # central finite differences (h = 1e-6) through the library's build + solve.
    # Their accuracy is set by the rounding of the two solves: with e_u the
    # solve's measured relative error on this workload (against the oracle
    # solution above), J carries an error up to 2 sum_m |r_m| e_u max|u|
    # (r = E u - u_obs), which the difference quotient divides by h; the
    # O(h^2) truncation is far below that.  A factor 4 covers the two
    # perturbed solves rounding differently from the unperturbed one.
    q0 = torch.tensor(inp["q"][0], device=DEV)
    h = 1e-6
    with torch.no_grad():
        _, u_q0 = J_of(q0)
        e_u = np.abs(u_q0[0].cpu().numpy() - u0).max() / np.abs(u0).max()
        r_obs = (observe(u_q0) - u_obs).abs().sum().item()
        tol_fd = 2 * r_obs * 4 * max(e_u, 1e-15) * u_q0.abs().max().item() / h
    say(f"[case] solve rel err {e_u:.2e}; finite-difference tolerance {tol_fd:.3e} "
        f"(|grad| max {np.abs(g0).max():.3e})")
    assert tol_fd < 1e-2 * np.abs(g0).max()   # the check is meaningful
    i, kk = np.unravel_index(np.argmax(np.abs(g0)), g0.shape)
    gsel = np.random.default_rng(23)
    dirs = []
    for (li, pk) in [(int(i), int(kk)),
                     (int(gsel.integers(g0.shape[0])), int(disc.Ii[gsel.integers(disc.n_i)])),
                     (int(gsel.integers(g0.shape[0])), int(disc.Ie[3]))]:
        d = np.zeros_like(g0)
        d[li, pk] = 1.0
        dirs.append((f"node ({li},{pk})", d))
    for b in range(2):   # smooth seeded bump directions, amplitude 1
        bp = W.draw_bumps(np.random.default_rng(300 + b), nbumps=1, amp=(1.0, 1.0), box=0.5, dim=2)
        dirs.append((f"bump {b}", W.eval_bumps(bp, pts, width=0.2)))
    for name, d in dirs:
        dt = torch.tensor(d, device=DEV)
        with torch.no_grad():
            fd = ((J_of(q0 + h * dt)[0] - J_of(q0 - h * dt)[0]) / (2 * h)).item()
        ad = float(np.sum(g0 * d))
        say(f"[case] fd {name}: {fd:.9e} vs adjoint {ad:.9e}")
        assert abs(fd - ad) < tol_fd


def test_autograd_source_and_boundary_gradients():
    import paper_2503_17535_amd as hp
    from paper_2503_17535_amd.autograd import solve as hsolve
    say("[case] autograd src / bdry gradients")
    d, p, L = 2, 10, 3
    t = hp.tree(d, L)
    pts = hp.leaf_points(t, p)
    bpts = hp.boundary_points(t, p)
    c, bd, src = W.helmholtz_inputs(pts, bpts, 5.0, 2)
    c_t = torch.tensor(c, device=DEV)
    bd_t = torch.tensor(bd, device=DEV, requires_grad=True)
    src_t = torch.tensor(src, device=DEV, requires_grad=True)
    w = torch.randn((2,) + pts.shape[:-1], dtype=torch.float64, device=DEV,
                    generator=torch.Generator(DEV).manual_seed(9))
    u = hsolve(t, p, c_t, bd_t, src_t)
    (w * u).sum().backward()
    op = hp.build(t, p, c_t)
    lb = torch.empty_like(bd_t)
    ls, lb = op.solve_adjoint(w.contiguous(), lam_bdry=lb)
    torch.cuda.synchronize()
    assert torch.equal(src_t.grad, ls) and torch.equal(bd_t.grad, lb)
    op.free()
