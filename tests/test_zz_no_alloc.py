"""The allocation-free solve (hps_solve_noalloc) against hps_solve and the
oracle.  It runs the same kernels on the library's static device workspace,
so its output must equal hps_solve's bit for bit; the oracle bar is the fp64
parity bar.  Two calls in a row on the same GPU, the second with a smaller
operator, fewer right-hand sides and no source: the second call must not
see the first call's leftovers in the shared workspace (the interface data
that a source-free solve needs at zero are cleared by a kernel)."""
import ctypes

import numpy as np
import pytest

from gpu_util import oracle_solve, rel_inf, rhs, say, var_coeffs
from oracle import hps as ohps

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-10


def _case(d, p, L, nrhs, seed, with_src, k=0.0):
    tree = ohps.Tree(d, L)
    disc = ohps.LeafDisc(d, p)
    pts = tree.leaf_points(disc)
    bpts = tree.root_boundary_points(disc)
    c = var_coeffs(pts, seed=seed, k=k)
    bd, src = rhs(pts, bpts, nrhs, seed=seed)
    ref = oracle_solve(d, p, L, c, bd, src if with_src else None)
    return c, bd, (src if with_src else None), ref


def _run(hp, d, p, L, nrhs, seed, with_src, k=0.0):
    c, bd, src, ref = _case(d, p, L, nrhs, seed, with_src, k)
    dev = torch.device("cuda:0")
    say(f"[case] noalloc d={d} p={p} L={L} nrhs={nrhs} src={with_src}")
    op = hp.build(hp.tree(d, L), p, torch.tensor(c, device=dev))
    b_d = torch.tensor(bd, device=dev)
    s_d = None if src is None else torch.tensor(src, device=dev)
    u_ref = op.solve(b_d, s_d)
    u_na = torch.full_like(u_ref, float("nan"))
    # through the C ABI directly
    rc = hp.lib().hps_solve_noalloc(op._h, ctypes.c_void_p(b_d.data_ptr()),
                                    None if s_d is None else ctypes.c_void_p(s_d.data_ptr()),
                                    ctypes.c_void_p(u_na.data_ptr()), nrhs, None)
    assert rc == hp.HPS_OK, hp.lib().hps_last_error().decode()
    torch.cuda.synchronize()
    op.free()
    same = torch.equal(u_na, u_ref)
    err = rel_inf(u_na.cpu().numpy(), ref)
    say(f"[case] bitwise equal to hps_solve: {same}; rel err vs oracle {err:.2e}")
    assert same
    assert err < TOL


def test_noalloc_two_calls_second_smaller():
    import paper_2503_17535_amd as hp
    # 20 rhs: two 16-column passes over the static workspace, with sources
    _run(hp, 2, 12, 4, 20, seed=3, with_src=True, k=4.0)
    # smaller operator, fewer rhs, no source
    _run(hp, 2, 8, 2, 3, seed=4, with_src=False)


def test_noalloc_3d():
    import paper_2503_17535_amd as hp
    _run(hp, 3, 6, 2, 2, seed=5, with_src=True)


def test_noalloc_rejects_operator_too_large():
    # depth 7, p = 16: its solve workspace (about 1 GiB) exceeds the static
    # array; the call must fail with a clear error and touch nothing
    import paper_2503_17535_amd as hp
    say("[case] noalloc size limit: 2D p=16 depth 7")
    t = hp.tree(2, 7)
    s = hp.sizes(t, 16)
    dev = torch.device("cuda:0")
    c = torch.zeros((s.n_leaves, s.n_terms, s.pts_per_leaf), dtype=torch.float64, device=dev)
    c[:, 0] = -1.0
    c[:, 2] = -1.0
    op = hp.build(t, 16, c)
    b = torch.zeros((1, s.n_root_bdry), dtype=torch.float64, device=dev)
    u = torch.zeros((1, s.n_leaves, s.pts_per_leaf), dtype=torch.float64, device=dev)
    with pytest.raises(hp.HPSError) as e:
        op.solve_noalloc(b, None, u)
    op.free()
    say(f"[case] rejected: {e.value}")
    assert e.value.code == hp.HPS_EINVAL and "static workspace" in str(e.value)
