"""Adaptive 3D path on the GPU (Section 4.2) against the adaptive oracle:
non-uniform merges across level jumps (element-wise parity), a uniform tree
against the uniform build, polynomial exactness, the refinement criterion and
the tree the GPU criterion builds, and the wavefront workload's accuracy."""
import numpy as np
import pytest

import workloads as W
from gpu_util import rel_inf, say, var_coeffs
from oracle import adaptive as A
from oracle import hps as ohps

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
TOL = 1e-10
DEV = "cuda:0"


def _jump_tree(lo=-1.0, hi=1.0):
    leaves = set(A.AdaptiveTree.uniform(1, lo, hi).leaves)
    for k in [(1, 0, 0, 0), (1, 1, 1, 1)]:
        leaves.remove(k)
        leaves.update(A.children(k))
    leaves.remove((2, 1, 1, 1))
    leaves.update(A.children((2, 1, 1, 1)))
    return A.AdaptiveTree(A.balance(leaves, lo, hi), lo, hi)


def _gpu_tree(ot):
    import paper_2503_17535_amd as hp
    return hp.AdaptiveTree(np.array(ot.leaves, dtype=np.int32), ot.lo, ot.hi)


def _rhs(pts, bpts, nrhs, seed):
    g = np.random.default_rng(500 + seed)
    bd = np.empty((nrhs, bpts.shape[0]))
    src = np.empty((nrhs,) + pts.shape[:-1])
    for r in range(nrhs):
        w = g.uniform(-2, 2, size=(3, 3))
        bd[r] = np.cos(bpts @ w[0]) + np.sin(bpts @ w[1])
        src[r] = np.exp(-np.sum((pts - 0.3 * w[2]) ** 2, axis=-1) * 4.0) * g.normal()
    return bd, src


def _parity(ot, p, nrhs, seed=0, with_src=True):
    import paper_2503_17535_amd as hp
    say(f"[case] adaptive p={p} leaves={len(ot.leaves)} levels={sorted({k[0] for k in ot.leaves})} nrhs={nrhs}")
    disc = ohps.LeafDisc(3, p)
    pts = ot.leaf_points(disc)
    c = var_coeffs(pts, seed, 0.0, True)
    oop = A.build(ot, p, c)
    bpts = A.root_boundary_points(oop)
    bd, src = _rhs(pts, bpts, nrhs, seed)
    ref = np.stack([A.solve(oop, bd[r], src[r] if with_src else None) for r in range(nrhs)])
    t = _gpu_tree(ot)
    assert np.abs(t.points(p, 2) - bpts).max() < 1e-14
    op = hp.build_adaptive(t, p, torch.tensor(c, device=DEV))
    assert op.root_D == A.root_D_size(ot, p)
    u = op.solve(torch.tensor(bd, device=DEV), torch.tensor(src, device=DEV) if with_src else None)
    err = rel_inf(u.cpu().numpy(), ref)
    say(f"[case] root D {op.root_D}, rel err vs oracle {err:.3e}, {op.nbytes / 2**20:.1f} MiB")
    op.free()
    return err


@pytest.mark.parametrize("p", [6, 7])
def test_parity_level_jumps(p):
    assert _parity(_jump_tree(), p, 3, seed=p) < TOL


def test_parity_no_source():
    assert _parity(_jump_tree(), 6, 1, seed=2, with_src=False) < TOL


def test_parity_refined_tree():
    """A tree the criterion refined around the wavefront, balanced."""
    leaves = A.refine_one(lambda x: W.wavefront_u(x), 6, 1e-2, 3)
    ot = A.AdaptiveTree(A.balance(leaves))
    assert len({k[0] for k in ot.leaves}) >= 2
    assert _parity(ot, 6, 2, seed=4) < TOL


def test_uniform_tree_equals_uniform_build():
    import paper_2503_17535_amd as hp
    say("[case] adaptive uniform depth 2, p=6 vs hps_build")
    p, L = 6, 2
    t = hp.AdaptiveTree.uniform(L, -1.0, 1.0)
    pts = hp.leaf_points(hp.tree(3, L), p)
    assert np.array_equal(pts, t.points(p, 0))
    bpts = hp.boundary_points(hp.tree(3, L), p)
    assert np.abs(t.points(p, 2) - bpts).max() < 1e-15
    c = torch.tensor(var_coeffs(pts, 1, 0.0, True), device=DEV)
    bd, src = _rhs(pts, bpts, 2, 1)
    bd, src = torch.tensor(bd, device=DEV), torch.tensor(src, device=DEV)
    ua = hp.build_adaptive(t, p, c).solve(bd, src).cpu().numpy()
    uu = hp.build(hp.tree(3, L), p, c).solve(bd, src).cpu().numpy()
    err = rel_inf(ua, uu)
    say(f"[case] adaptive vs uniform operator {err:.3e}")
    assert err < 1e-12


def test_polynomial_exact_across_level_jumps():
    import paper_2503_17535_amd as hp
    p = 8
    say(f"[case] adaptive polynomial p={p}")
    ot = _jump_tree()
    t = _gpu_tree(ot)
    pts = t.points(p, 0)
    bpts = t.points(p, 2)
    # u of per-variable degree p - 3 under -Laplace: exact for every panel map
    from numpy.polynomial import polynomial as npoly
    cf = [np.array([0.2, -0.3, 0.1, 0.05, 0.0, 0.4 + 0.1 * a]) for a in range(3)]

    def u_of(x):
        v = [npoly.polyval(x[..., a], cf[a]) for a in range(3)]
        return v[0] * v[1] * v[2]

    def lap_of(x):
        v = [npoly.polyval(x[..., a], cf[a]) for a in range(3)]
        d2 = [npoly.polyval(x[..., a], npoly.polyder(cf[a], 2)) for a in range(3)]
        return d2[0] * v[1] * v[2] + v[0] * d2[1] * v[2] + v[0] * v[1] * d2[2]

    c = W.coeffs_poisson(pts)
    op = hp.build_adaptive(t, p, torch.tensor(c, device=DEV))
    u = op.solve(torch.tensor(u_of(bpts)[None], device=DEV), torch.tensor(-lap_of(pts)[None], device=DEV))
    ue = u_of(pts)
    err = np.abs(u.cpu().numpy()[0] - ue).max() / np.abs(ue).max()
    say(f"[case] rel error vs exact polynomial {err:.3e}")
    assert err < 1e-11


def test_large_root_polynomial_exact():
    """p = 12 wavefront tree (root D = 8400, beyond 8192: the widest
    Gauss-Jordan panel instance): a polynomial of per-variable degree p - 3
    is reproduced to rounding."""
    import paper_2503_17535_amd as hp
    p = 12
    funcs = [lambda x: W.wavefront_u(x), lambda x: W.wavefront_f(x)]
    t = hp.adaptive_tree(funcs, p, 1e-5, 3)
    pts, bpts = t.points(p, 0), t.points(p, 2)
    from numpy.polynomial import polynomial as npoly
    cf = [np.array([0.2, -0.3, 0.1, 0.05] + [0.0] * (p - 7) + [0.4 + 0.1 * a]) for a in range(3)]
    vals = lambda x: [npoly.polyval(x[..., a], cf[a]) for a in range(3)]
    d2s = lambda x: [npoly.polyval(x[..., a], npoly.polyder(cf[a], 2)) for a in range(3)]
    v, d2 = vals(pts), d2s(pts)
    lap = d2[0] * v[1] * v[2] + v[0] * d2[1] * v[2] + v[0] * v[1] * d2[2]
    vb = vals(bpts)
    op = hp.build_adaptive(t, p, torch.tensor(W.coeffs_poisson(pts), device=DEV))
    say(f"[case] adaptive p={p} leaves={t.n_leaves} root D {op.root_D}")
    assert op.root_D > 8192
    u = op.solve(torch.tensor((vb[0] * vb[1] * vb[2])[None], device=DEV), torch.tensor(-lap[None], device=DEV))
    ue = v[0] * v[1] * v[2]
    err = np.abs(u.cpu().numpy()[0] - ue).max() / np.abs(ue).max()
    op.free()
    say(f"[case] rel error vs exact polynomial {err:.3e}")
    assert err < 1e-10


def test_refinement_check_matches_oracle_tree():
    """The tree built with the GPU criterion equals the oracle's (same
    functions, tolerance, level cap): bit-exact integer output."""
    import paper_2503_17535_amd as hp
    p, eps, cap = 6, 1e-3, 4
    say(f"[case] adaptive_tree p={p} eps={eps} cap={cap}")
    funcs = [lambda x: W.wavefront_u(x), lambda x: W.wavefront_f(x)]
    t = hp.adaptive_tree(funcs, p, eps, cap)
    ot = A.adaptive_tree(funcs, p, eps, cap)
    say(f"[case] leaves {t.n_leaves} (oracle {len(ot.leaves)})")
    assert [tuple(int(v) for v in k) for k in t.leaves] == ot.leaves


def test_refinement_check_flags():
    import paper_2503_17535_amd as hp
    p = 7
    t = _gpu_tree(_jump_tree(0.0, 1.0))
    x0, x1 = t.points(p, 0), t.points(p, 1)
    f = lambda x: np.exp(-30.0 * np.sum((x - 0.3) ** 2, axis=-1)) + 0.1 * x[..., 0] ** 6
    f0, f1 = f(x0), f(x1)
    L8 = A.child_interp(p)
    err = np.array([np.abs(f1[i].reshape(-1) - L8 @ f0[i]).max() for i in range(t.n_leaves)])
    fn = np.abs(f0).max()
    # tolerances away from every leaf's ratio, so rounding cannot flip a flag
    ratios = np.unique(err / fn)
    gap = int(np.argmax(ratios[1:] / ratios[:-1]))          # widest gap between distinct ratios
    mid = np.sqrt(ratios[gap] * ratios[gap + 1])
    assert ratios[gap + 1] / ratios[gap] > 1.5
    for eps in (ratios[0] / 2, mid, ratios[-1] * 2):
        flags = hp.adaptive_check(p, torch.tensor(f0, device=DEV), torch.tensor(f1, device=DEV), eps)
        assert np.array_equal(flags, (~(err < eps * fn)).astype(np.int32))


def _wavefront_error(op_build, pts, bpts):
    u = op_build.solve(torch.tensor(W.wavefront_u(bpts)[None], device=DEV),
                       torch.tensor(W.wavefront_f(pts)[None], device=DEV)).cpu().numpy()[0]
    ue = W.wavefront_u(pts)
    return np.abs(u - ue).max() / np.abs(ue).max()


def test_wavefront_adaptive_beats_uniform():
    """Section 4.2's comparison on the wavefront problem (p = 8): the adaptive
    tree (eps = 1e-4, finest level 4) has a smaller root D than the uniform
    depth-3 tree and a smaller error against the exact solution."""
    import paper_2503_17535_amd as hp
    p = 8
    funcs = [lambda x: W.wavefront_u(x), lambda x: W.wavefront_f(x)]
    t = hp.adaptive_tree(funcs, p, 1e-4, 4)
    pts, bpts = t.points(p, 0), t.points(p, 2)
    op = hp.build_adaptive(t, p, torch.tensor(W.coeffs_poisson(pts), device=DEV))
    err_a, D_a = _wavefront_error(op, pts, bpts), op.root_D
    op.free()
    tu = hp.tree(3, 3, 0.0, 1.0)
    pu, bu = hp.leaf_points(tu, p), hp.boundary_points(tu, p)
    opu = hp.build(tu, p, torch.tensor(W.coeffs_poisson(pu), device=DEV))
    err_u, D_u = _wavefront_error(opu, pu, bu), hp.sizes(tu, p).root_D
    opu.free()
    say(f"[case] wavefront p={p}: adaptive {t.n_leaves} leaves, root D {D_a}, rel err {err_a:.3e}; "
        f"uniform 512 leaves, root D {D_u}, rel err {err_u:.3e}")
    assert D_a < D_u and err_a < err_u


def test_unsupported_calls_are_refused():
    import ctypes

    import paper_2503_17535_amd as hp
    say("[case] adaptive operator: unsupported calls")
    p = 5
    t = _gpu_tree(_jump_tree())
    pts = t.points(p, 0)
    op = hp.build_adaptive(t, p, torch.tensor(W.coeffs_poisson(pts), device=DEV))
    w = torch.zeros((1, t.n_leaves, p ** 3), dtype=torch.float64, device=DEV)
    bd = torch.zeros((1, op.n_root_bdry), dtype=torch.float64, device=DEV)
    L = hp.lib()
    st = hp._stream_ptr(None)
    ptr = ctypes.c_void_p(w.data_ptr())
    assert L.hps_solve_adjoint(op._h, ptr, ptr, None, 1, st) == hp.HPS_EUNSUPPORTED
    assert L.hps_solve_noalloc(op._h, ctypes.c_void_p(bd.data_ptr()), None, ptr, 1, st) == hp.HPS_EUNSUPPORTED
    assert L.hps_coeff_grad(op._h, ptr, ptr, 1, ptr, st) == hp.HPS_EUNSUPPORTED
    assert L.hps_solve(op._h, ctypes.c_void_p(bd.data_ptr()), None, ptr, 1, hp.FP32_REFINED, st) != hp.HPS_OK
    u = op.solve(bd)
    assert torch.all(u == 0.0)  # zero data, zero source: zero solution
    op.free()
