"""Allocator callback (hps_set_allocator) on the GPU: operators built with
PyTorch's caching allocator give bitwise the same solutions as operators in
the library's pool, their bytes show up in torch's accounting and go back on
free; an allocator with a byte budget makes a build that does not fit return
HPS_ENOMEM with every block it had taken returned."""
import numpy as np
import pytest

from gpu_util import rhs, say, var_coeffs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DEV = "cuda:0"


def _inputs(hp, L, p):
    t = hp.tree(2, L)
    pts = hp.leaf_points(t, p)
    bpts = hp.boundary_points(t, p)
    c = var_coeffs(pts, seed=4, k=6.0)
    bd, src = rhs(pts, bpts, 3, seed=4)
    return t, torch.tensor(c, device=DEV), torch.tensor(bd, device=DEV), torch.tensor(src, device=DEV)


def test_torch_allocator_same_results_and_accounting():
    import paper_2503_17535_amd as hp
    say("[case] torch caching allocator")
    t, c, bd, src = _inputs(hp, 4, 12)
    ref_op = hp.build(t, 12, c)
    ref = ref_op.solve(bd, src)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    hp.use_torch_allocator()
    try:
        op = hp.build(t, 12, c)
        during = torch.cuda.memory_allocated()
        u = op.solve(bd, src)
        torch.cuda.synchronize()
        say(f"[case] torch allocated +{(during - before) / 2**20:.1f} MiB for an operator of "
            f"{op.nbytes / 2**20:.1f} MiB resident")
        assert during - before >= op.nbytes
        assert torch.equal(u, ref)
        op.free()
        del u
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() <= before + (1 << 20)
    finally:
        hp.use_torch_allocator(False)
    ref_op.free()


def test_allocator_budget_gives_enomem():
    import paper_2503_17535_amd as hp
    say("[case] allocator with a byte budget")
    t, c, bd, src = _inputs(hp, 4, 12)
    state = {"out": 0, "budget": 8 << 20, "refused": 0}

    def alloc(n):
        if state["out"] + n > state["budget"]:
            state["refused"] += 1
            return None
        state["out"] += n
        return torch.cuda.caching_allocator_alloc(n)

    def free(p, n):
        state["out"] -= n
        torch.cuda.caching_allocator_delete(p)

    hp.set_allocator(alloc, free)
    try:
        with pytest.raises(hp.HPSError) as e:
            hp.build(t, 12, c)
        assert e.value.code == hp.HPS_ENOMEM
        assert state["refused"] >= 1 and state["out"] == 0
        state["budget"] = 1 << 40
        op = hp.build(t, 12, c)
        u = op.solve(bd, src)
        torch.cuda.synchronize()
        assert state["out"] > 0
        op.free()
        assert state["out"] == 0
        assert np.isfinite(u.cpu().numpy()).all()
    finally:
        hp.set_allocator(None, None)
