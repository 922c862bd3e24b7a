"""Subtree recomputation (Section 4.1, Algorithm "Subtree recomputation
strategy") on the GPU.

* small trees: the solve of an operator that keeps only the top levels
  resident and rebuilds every subtree on demand, against the oracle
  (rel. l_inf <= 1e-10, the solver's fp64 bar) and against the fully resident
  operator's solve, with and without sources, for subtree depths 1 and
  depth - 1, a Helmholtz-like operator and more than 16 right-hand sides;
* adjoint checkpointing: the transposed solve of such an operator against
  the oracle's adjoint (1e-10), and it and the coefficient gradient against
  the resident operator's;
* a 2D p = 16 tree of depth 8 (16.8M unknowns) whose resident operator needs
  three times a 12 GiB device-memory budget: built with 5-level subtrees,
  the library's device memory stays inside the budget through build and
  solve; the solve equals the resident operator's (which fits the device,
  not the budget) to 1e-11, and reproduces a degree-5 polynomial solution of
  a variable-coefficient problem to rounding.  The discretization is exact
  for traces of degree <= p - 3, so a wrong subtree datum would show at
  O(1); what remains is rounding amplified by the conditioning of the
  discrete operator, which grows like h^-2: measured 1.7e-11, 6.9e-11,
  2.8e-10, 1.1e-9 at depths 5-8 for both operators, so the bar is
  1e-13 * 4^depth (about six times the measured error).
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import oracle_solve, rel_inf, rhs, say, var_coeffs
from oracle import hps as ohps

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DEV = "cuda:0"
TOL = 1e-10


def _small(p, L, sd, nrhs, seed=0, k=0.0, with_src=True):
    import paper_2503_17535_amd as hp
    say(f"[case] subtrees p={p} L={L} subtree_depth={sd} nrhs={nrhs} k={k} src={with_src}")
    tree = ohps.Tree(2, L)
    disc = ohps.LeafDisc(2, p)
    pts = tree.leaf_points(disc)
    bpts = tree.root_boundary_points(disc)
    c = var_coeffs(pts, seed, k, mixed=True)
    bd, src = rhs(pts, bpts, nrhs, seed)
    if not with_src:
        src = None
    ref = oracle_solve(2, p, L, c, bd, src)
    t = hp.tree(2, L)
    ct = torch.tensor(c, device=DEV)
    bdt = torch.tensor(bd, device=DEV)
    srct = None if src is None else torch.tensor(src, device=DEV)
    op = hp.build_subtrees(t, p, ct, sd)
    u = op.solve(bdt, srct)
    u2 = op.solve(bdt, srct)          # the second solve rebuilds the subtrees again
    full = hp.build(t, p, ct)
    uf = full.solve(bdt, srct)
    torch.cuda.synchronize()
    err = rel_inf(u.cpu().numpy(), ref)
    dif = rel_inf(u.cpu().numpy(), uf.cpu().numpy())
    say(f"[case] vs oracle {err:.3e}, vs resident operator {dif:.3e}; "
        f"resident bytes {op.nbytes / 2**20:.1f} MiB vs {full.nbytes / 2**20:.1f} MiB")
    assert torch.equal(u, u2)
    assert err < TOL
    assert dif < 1e-11
    op.free()
    full.free()


@pytest.mark.parametrize("p,L,sd,nrhs", [(8, 3, 1, 2), (12, 4, 2, 3), (10, 4, 3, 1), (6, 3, 2, 18)])
def test_subtrees_small_against_oracle(p, L, sd, nrhs):
    _small(p, L, sd, nrhs)


def test_subtrees_no_source():
    _small(8, 4, 2, 2, with_src=False)


def test_subtrees_helmholtz_like_p16():
    _small(16, 4, 2, 2, k=10.0)


def test_subtree_operator_rejects_other_solves():
    import paper_2503_17535_amd as hp
    say("[case] subtree operator: unsupported solves")
    t = hp.tree(2, 3)
    s = hp.sizes(t, 8)
    pts = hp.leaf_points(t, 8)
    c = torch.tensor(var_coeffs(pts), device=DEV)
    op = hp.build_subtrees(t, 8, c, 1)
    bd = torch.zeros((1, s.n_root_bdry), dtype=torch.float64, device=DEV)
    u = torch.zeros((1, s.n_leaves, s.pts_per_leaf), dtype=torch.float64, device=DEV)
    for call in (lambda: op.solve_noalloc(bd, None, u), lambda: op.solve(bd, None, precision=hp.FP32_REFINED)):
        with pytest.raises(hp.HPSError) as e:
            call()
        assert e.value.code in (hp.HPS_EUNSUPPORTED, hp.HPS_EINVAL)
    b = hp.Batcher()
    with pytest.raises(hp.HPSError) as e:
        b.solve([(op, [bd[0]], None, [u[0]])])
    assert e.value.code == hp.HPS_EUNSUPPORTED
    b.free()
    op.free()


@pytest.mark.parametrize("p,L,sd,nrhs,k", [(8, 3, 1, 2, 0.0), (12, 4, 2, 3, 10.0), (7, 4, 3, 18, 2.0)])
def test_subtrees_adjoint_and_gradient(p, L, sd, nrhs, k):
    """Adjoint checkpointing: the transposed solve of a recomputing operator
    (every subtree rebuilt twice) against the oracle's adjoint, and it and the
    coefficient gradient against the resident operator's."""
    import paper_2503_17535_amd as hp
    from oracle import adjoint as A
    say(f"[case] subtree adjoint p={p} L={L} subtree_depth={sd} nrhs={nrhs} k={k}")
    tree = ohps.Tree(2, L)
    disc = ohps.LeafDisc(2, p)
    pts = tree.leaf_points(disc)
    c = var_coeffs(pts, seed=3, k=k)
    w = np.random.default_rng(21).normal(size=(nrhs,) + pts.shape[:-1])
    op_o = ohps.build(tree, p, c)
    ref = [A.hps_adjoint(op_o, w[r]) for r in range(nrhs)]
    t = hp.tree(2, L)
    ct = torch.tensor(c, device=DEV)
    wt = torch.tensor(w, device=DEV)
    op = hp.build_subtrees(t, p, ct, sd)
    full = hp.build(t, p, ct)
    outs = []
    for o in (op, full):
        lb = torch.empty((nrhs, o.sizes.n_root_bdry), dtype=torch.float64, device=DEV)
        ls, lb = o.solve_adjoint(wt, lam_bdry=lb)
        u = o.solve(torch.tensor(rhs(pts, tree.root_boundary_points(disc), nrhs)[0], device=DEV))
        grad = o.coeff_grad(u, ls)
        outs.append((ls, lb, grad))
    torch.cuda.synchronize()
    ls, lb, grad = (x.cpu().numpy() for x in outs[0])
    es = max(np.abs(ls[r] - ref[r][0]).max() / np.abs(ref[r][0]).max() for r in range(nrhs))
    eb = max(np.abs(lb[r] - ref[r][1]).max() / np.abs(ref[r][1]).max() for r in range(nrhs))
    dl = max((outs[0][i] - outs[1][i]).abs().max().item() / outs[1][i].abs().max().item() for i in range(3))
    say(f"[case] lam_src rel err {es:.3e}  lam_bdry rel err {eb:.3e}; vs resident operator {dl:.3e}")
    assert es < TOL and eb < TOL
    assert dl < 1e-11
    assert np.all(ls[:, :, disc.Ie] == 0.0)
    op.free()
    full.free()


def test_subtrees_beyond_memory_budget_depth8_p16():
    import paper_2503_17535_amd as hp
    budget = 12 << 30
    L, p, sd = 8, 16, 5
    t = hp.tree(2, L)
    full_bytes = hp.footprint(t, p)
    say(f"[case] depth {L} p {p}: resident operator {full_bytes / 2**30:.1f} GiB, budget {budget / 2**30:.0f} GiB")
    assert full_bytes > 2.5 * budget
    pts = hp.leaf_points(t, p)
    bpts = hp.boundary_points(t, p)
    c, f, g, uex = W.poly5_problem(pts, bpts)
    ct = torch.tensor(c, device=DEV)
    ft = torch.tensor(f[None], device=DEV)
    gt = torch.tensor(g[None], device=DEV)
    del c, f
    full = hp.build(t, p, ct)
    uf = full.solve(gt, ft)
    full.free()
    torch.cuda.synchronize()
    base, _ = hp.mem_stats(reset_peak=True)
    op = hp.build_subtrees(t, p, ct, sd)
    u = op.solve(gt, ft)
    torch.cuda.synchronize()
    used, peak = hp.mem_stats()
    say(f"[case] library device memory: peak {(peak - base) / 2**30:.2f} GiB over build and solve "
        f"(resident {op.nbytes / 2**30:.2f} GiB)")
    assert peak - base <= budget
    scale = np.abs(uex).max()
    err = np.abs(u[0].cpu().numpy() - uex).max() / scale
    err_f = np.abs(uf[0].cpu().numpy() - uex).max() / scale
    dif = (u - uf).abs().max().item() / scale
    say(f"[case] polynomial solution: rel l_inf error {err:.3e} (resident operator {err_f:.3e}), "
        f"difference {dif:.3e}")
    assert dif < 1e-11
    assert err < 1e-13 * 4.0**L
    op.free()


def test_subtrees_autograd_checkpointing():
    """torch.autograd through a recomputing build: the backward pass rebuilds
    the subtrees' factors instead of storing them; the gradients with respect
    to the coefficients, the source and the boundary data equal those of the
    resident build to rounding."""
    import paper_2503_17535_amd as hp
    from paper_2503_17535_amd.autograd import solve as hsolve
    say("[case] autograd with subtree recomputation")
    p, L = 12, 4
    t = hp.tree(2, L)
    pts = hp.leaf_points(t, p)
    bpts = hp.boundary_points(t, p)
    c, bd, src = W.helmholtz_inputs(pts, bpts, 8.0, 2)
    w = torch.randn((2,) + pts.shape[:-1], dtype=torch.float64, device=DEV,
                    generator=torch.Generator(DEV).manual_seed(9))
    grads = []
    for sd in (0, 2):
        c_t = torch.tensor(c, device=DEV, requires_grad=True)
        bd_t = torch.tensor(bd, device=DEV, requires_grad=True)
        src_t = torch.tensor(src, device=DEV, requires_grad=True)
        u = hsolve(t, p, c_t, bd_t, src_t, subtree_depth=sd)
        (w * u).sum().backward()
        grads.append((u.detach(), c_t.grad, bd_t.grad, src_t.grad))
    torch.cuda.synchronize()
    for a, b in zip(*grads):
        rel = (a - b).abs().max().item() / b.abs().max().item()
        assert rel < 1e-11, rel
