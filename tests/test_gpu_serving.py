"""Batched multi-operator solve and the continuous-batching server on the GPU.

* a batch over operators of different depth and p, with several right-hand
  sides per operator and mixed zero / non-zero sources, equals the
  single-operator solve of every item exactly (the arithmetic of every output
  entry is the same), and matches the oracle (rel. l_inf <= 1e-10);
* every request served in the mix equals the same request solved alone, in
  fp64 and in the mixed-precision mode (whose results also meet 1e-8 against
  the oracle), and in fp64 batches of different operator classes overlap on
  the device;
* the serving workload (8 resident operators, depths 4-7, p 12/16, 4096
  requests at 2000/s) completes with every request accounted for.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import oracle_solve, rel_inf, say
from oracle import hps as ohps

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DEV = "cuda:0"


def _op_inputs(depth, p, k, nrhs, op_seed):
    import paper_2503_17535_amd as hp
    t = hp.tree(2, depth)
    pts = hp.leaf_points(t, p)
    bpts = hp.boundary_points(t, p)
    c, bd, src = W.helmholtz_inputs(pts, bpts, k, nrhs, config=4, op_seed=op_seed)
    return t, c, bd, src


def test_batch_equals_single_solves_and_oracle():
    import paper_2503_17535_amd as hp
    say("[case] batched solve vs single solves")
    specs = [(3, 12, 10.0, 3), (4, 16, 20.0, 2), (2, 8, 5.0, 5), (5, 12, 20.0, 1)]
    ops, data = [], []
    for s, (L, p, k, nr) in enumerate(specs):
        t, c, bd, src = _op_inputs(L, p, k, nr, s)
        ops.append(hp.build(t, p, torch.tensor(c, device=DEV)))
        data.append((c, torch.tensor(bd, device=DEV), torch.tensor(src, device=DEV)))
    # item 1: no sources at all; item 2: rhs 1 and 3 without source
    items, outs = [], []
    for s, (op, (c, bd, src)) in enumerate(zip(ops, data)):
        nr = bd.shape[0]
        sl = None if s == 1 else [None if (s == 2 and j in (1, 3)) else src[j] for j in range(nr)]
        u = [torch.empty_like(src[0]) for _ in range(nr)]
        items.append((op, [bd[j] for j in range(nr)], sl, u))
        outs.append(u)
    b = hp.Batcher()
    b.solve(items)
    torch.cuda.synchronize()
    for s, (op, (c, bd, src)) in enumerate(zip(ops, data)):
        nr = bd.shape[0]
        if s == 1:
            ref = op.solve(bd, None)
        else:
            srcz = src.clone()
            if s == 2:
                srcz[1].zero_()
                srcz[3].zero_()
            ref = op.solve(bd, srcz)
        got = torch.stack(outs[s])
        assert torch.equal(got, ref), (s, (got - ref).abs().max().item())
    # oracle parity of two items
    for s in (0, 3):
        L, p, k, nr = specs[s]
        c, bd, src = data[s]
        ref = oracle_solve(2, p, L, c, bd.cpu().numpy(), src.cpu().numpy())
        err = rel_inf(torch.stack(outs[s]).cpu().numpy(), ref)
        say(f"[case] batched item {s} vs oracle: rel err {err:.3e}")
        assert err < 1e-10
    b.free()
    for op in ops:
        op.free()


def _serving_setup(specs, pool, seed_base=0, flags=0):
    import paper_2503_17535_amd as hp
    ops, pools = [], []
    for s, (L, p, k) in enumerate(specs):
        t, c, bd, src = _op_inputs(L, p, k, pool, seed_base + s)
        ops.append(hp.build(t, p, torch.tensor(c, device=DEV), flags=flags))
        pools.append((torch.tensor(bd, device=DEV), torch.tensor(src, device=DEV)))
    return ops, pools


def _overlapping_classes(trace):
    """Pairs of batches of different classes whose device intervals overlap."""
    n = 0
    for i, (ca, a0, a1) in enumerate(trace):
        for cb, b0, b1 in trace[i + 1:]:
            if ca != cb and a0 < b1 and b0 < a1:
                n += 1
    return n


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_serving_results_alone_equal_in_mix(precision):
    import paper_2503_17535_amd as hp
    from paper_2503_17535_amd.serve import Request, Server, latency_stats
    say(f"[case] serving ({precision}): alone == in the mix")
    specs = W.SERVING_OPS[:6]           # depths 4-6: two classes
    pool = 4
    flags = hp.FLAG_FP32_COPY if precision == "fp32_refined" else 0
    ops, pools = _serving_setup(specs, pool, flags=flags)
    t, opi, rhs = W.serving_arrivals(600, 4000.0, len(specs), pool)
    reqs = []
    for i in range(len(t)):
        bd, src = pools[opi[i]]
        # fp64: a third of the requests carry no source
        use_src = precision != "fp64" or (i % 3) != 0
        reqs.append(Request(op=int(opi[i]), bdry=bd[rhs[i]], src=src[rhs[i]] if use_src else None,
                            t_arrival=float(t[i])))
    srv = Server(ops, precision=precision)
    srv.run(reqs)
    torch.cuda.synchronize()
    st = latency_stats(reqs)
    ov = _overlapping_classes(srv.trace)
    say(f"[case] served {st['requests']} requests in {len(srv.batches)} batches "
        f"(mean {np.mean(srv.batches):.1f}), {len(srv.classes)} classes, {ov} overlapping batch pairs; "
        f"p50 {st['p50_ms']:.3f} ms p99 {st['p99_ms']:.3f} ms")
    assert len(srv.classes) == 2
    assert all(r.t_done >= r.t_admit >= r.t_arrival for r in reqs)
    assert max(srv.batches) > 1          # requests were batched together
    if precision == "fp64":
        # batches of the two classes ran at the same time (the refined mode
        # issues one mixed-precision solve per operator and batch, a few
        # hundred small launches, so at this size the host's launch rate and
        # not the device decides whether two batches meet)
        assert ov > 0
    prec = hp.FP32_REFINED if precision == "fp32_refined" else hp.FP64
    for r in reqs:
        alone = ops[r.op].solve(r.bdry[None].contiguous(), None if r.src is None else r.src[None].contiguous(),
                                precision=prec)
        assert torch.equal(alone[0], r.u), r
    if precision == "fp32_refined":
        # the refined results against the oracle (two operators, one request each)
        for k in (0, 3):
            r = next(x for x in reqs if x.op == k)
            L, p, kw = specs[k]
            tt, c, _, _ = _op_inputs(L, p, kw, 1, k)
            ref = oracle_solve(2, p, L, c, r.bdry[None].cpu().numpy(), r.src[None].cpu().numpy())
            err = rel_inf(r.u[None].cpu().numpy(), ref)
            say(f"[case] refined request on operator {k} vs oracle: rel err {err:.2e}")
            assert err < 1e-8
    srv.free()
    for op in ops:
        op.free()


def test_serving_workload_completes():
    from paper_2503_17535_amd.serve import Request, Server, latency_stats
    say("[case] serving workload: 8 operators, 4096 requests at 2000/s")
    pool = 4
    ops, pools = _serving_setup(W.SERVING_OPS, pool)
    t, opi, rhs = W.serving_arrivals(4096, 2000.0, len(ops), pool)
    reqs = [Request(op=int(opi[i]), bdry=pools[opi[i]][0][rhs[i]], src=pools[opi[i]][1][rhs[i]],
                    t_arrival=float(t[i])) for i in range(len(t))]
    srv = Server(ops)
    srv.run(reqs)
    torch.cuda.synchronize()
    st = latency_stats(reqs)
    say(f"[case] {st}")
    assert st["requests"] == 4096 and np.isfinite(st["p99_ms"])
    # a sample of requests against their solo solves
    for r in reqs[::256]:
        alone = ops[r.op].solve(r.bdry[None].contiguous(), r.src[None].contiguous())
        assert torch.equal(alone[0], r.u)
    srv.free()
    for op in ops:
        op.free()
