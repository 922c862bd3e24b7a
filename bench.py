#!/usr/bin/env python3
"""Throughput of the HPS hot path on one MI355X.

Workload (the configuration the headline metric is quoted on): 2D
variable-coefficient Helmholtz  -Lap u - k^2 (1 + q(x)) u = f  on [-1, 1]^2,
k = 40, q = 8 seeded Gaussian bumps (amplitude U(0, 0.5), width 0.1), uniform
quadtree of depth 6 (4096 leaves), p = 16, fp64, 16 right-hand sides (Fourier
boundary data + one Gaussian source bump each).  Inputs are synthetic, seeded
(``workloads``), and resident in HBM before timing starts.

One step = build (leaf stage + all merge levels) + one 16-rhs solve (upward
source pass + downward pass) + release of the operator.  ``value`` is leaves
per second of whole steps; build-only leaves/s and solves/s are reported
beside it from HIP events on the stream the library runs on.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "HPS build leaves/s + solves/s at rel.err<=1e-10; serving p99 latency"
K_WAVE, DEPTH, P, NRHS = 40.0, 6, 16, 16

# MI355X published peaks used for roofline fractions
PEAK_FP64_TFLOPS = 78.6      # fp64 vector and fp64 matrix (256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz)
PEAK_HBM_GBS = 8000.0


def leaf_flops(p: int) -> float:
    """Algorithmic flops of one 2D leaf in the fused leaf kernel: LU of
    L_ii (n_i = (p-2)^2) with partial pivoting, (2/3) n_i^3, plus the forward
    and back substitution of the n_b = 4(p-2) columns of L_ie P, 2 n_i^2 n_b."""
    ni, nb = (p - 2) ** 2, 4 * (p - 2)
    return (2.0 / 3.0) * ni ** 3 + 2.0 * ni * ni * nb


def cpu_baseline(seconds_budget: float = 30.0):
    """The oracle (plain NumPy/SciPy) on a bounded sample of the workload:
    one quadrant subtree of depth 5 (1024 leaves, same p, k and inputs), build
    + 16 solves, scaled to leaves/s."""
    import numpy as np
    import workloads as W
    from oracle import hps as ohps
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    depth = DEPTH - 1
    tree = ohps.Tree(2, depth, -1.0, 0.0)          # the SW quadrant of [-1,1]^2
    disc = ohps.LeafDisc(2, P)
    pts = tree.leaf_points(disc)
    bpts = tree.root_boundary_points(disc)
    c, bd, src = W.helmholtz_inputs(pts, bpts, K_WAVE, NRHS)
    t0 = time.perf_counter()
    op = ohps.build(tree, P, c)
    t1 = time.perf_counter()
    for r in range(NRHS):
        ohps.solve(op, bd[r], src[r])
    t2 = time.perf_counter()
    nl = tree.n_leaves
    return {"value": nl / (t2 - t0), "unit": "leaves/s", "cores": int(threads), "kind": "oracle",
            "sample": f"oracle build + {NRHS} solves of one depth-{depth} quadrant subtree "
                      f"({nl} leaves, p={P}, k={K_WAVE:g}); build {t1 - t0:.2f}s, solves {t2 - t1:.2f}s",
            "build_leaves_per_s": nl / (t1 - t0), "solves_per_s": NRHS / (t2 - t1)}


def _leaf_source_hash():
    """sha256 prefix over the sources of the leaf kernel (kernel + helpers)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("leaf2d.hip", "dpp.hpp", "common.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2503_17535_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the leaf kernel from its committed rocprofv3
    counter summary, if that summary was taken on the current sources."""
    prof = os.path.join(ROOT, "profiles", "leaf2d_factor_kernel_p16_hbm_counters.md")
    try:
        txt = open(prof).read()
        if f"sources sha256 prefix: {_leaf_source_hash()}" not in txt:
            return None
        for line in txt.splitlines():
            if line.startswith("traffic_bytes_per_launch:"):
                return float(line.split(":")[1])
    except OSError:
        pass
    return None


def _median_ms(fn, reps=5):
    import numpy as np
    import torch
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def solve_rates(hp, t, c_d, b_d, s_d, sz):
    """Solve-only rates of one resident operator: 16 and 1 right-hand sides
    (median of 5 after a warm-up)."""
    op = hp.build(t, P, c_d)
    u16 = op.solve(b_d, s_d)
    ms16 = _median_ms(lambda: op.solve(b_d, s_d, out=u16))
    b1, s1 = b_d[:1].contiguous(), s_d[:1].contiguous()
    u1 = op.solve(b1, s1)
    ms1 = _median_ms(lambda: op.solve(b1, s1, out=u1))
    op.free()
    return {"solve16_ms": ms16, "solves_per_s_nrhs16": NRHS * 1e3 / ms16,
            "solve1_ms": ms1, "solves_per_s_nrhs1": 1e3 / ms1}


def refined_solve(hp, t, c_d, b_d, s_d):
    """Mixed-precision solve of the same workload (fp32 operator copies, fp64
    residual refinement): time and the max relative difference to the fp64
    solve of the same operator (the tests check both against the oracle)."""
    import torch
    op = hp.build(t, P, c_d, flags=hp.FLAG_FP32_COPY)
    u64 = op.solve(b_d, s_d)
    sweeps = op.refine_sweeps()
    u = op.solve(b_d, s_d, precision=hp.FP32_REFINED)
    ms = _median_ms(lambda: op.solve(b_d, s_d, out=u, precision=hp.FP32_REFINED))
    diff = ((u - u64).abs().amax(dim=(1, 2)) / u64.abs().amax(dim=(1, 2))).max().item()
    op.free()
    torch.cuda.synchronize()
    return {"sweeps": sweeps, "solve16_ms": ms, "solves_per_s": NRHS * 1e3 / ms,
            "max_rel_diff_to_fp64": diff}


def serving(hp, W, n_req=4096, rate=2000.0, pool=4):
    """Continuous-batching serving: 8 resident Helmholtz operators (depths 4-7,
    p 12/16, k 10-40), 4096 requests with exponential inter-arrival times at
    2000/s replayed against the wall clock, each one right-hand side (Fourier
    boundary data + one source bump) for a uniformly chosen operator; fp64.
    Latency = device completion - scheduled arrival."""
    import numpy as np
    import torch
    from paper_2503_17535_amd.serve import Request, Server, latency_stats
    dev = torch.device("cuda:0")
    ops, pools = [], []
    for k, (L, p, kw) in enumerate(W.SERVING_OPS):
        tt = hp.tree(2, L)
        pts = hp.leaf_points(tt, p)
        bpts = hp.boundary_points(tt, p)
        c, bd, src = W.helmholtz_inputs(pts, bpts, kw, pool, config=4, op_seed=k)
        ops.append(hp.build(tt, p, torch.tensor(c, device=dev)))
        pools.append((torch.tensor(bd, device=dev), torch.tensor(src, device=dev)))
    resident = sum(op.nbytes for op in ops)
    ta, opi, rhs = W.serving_arrivals(n_req, rate, len(ops), pool)
    # warm-up pass (not measured)
    warm = [Request(op=i % len(ops), bdry=pools[i % len(ops)][0][0], src=pools[i % len(ops)][1][0],
                    t_arrival=0.0) for i in range(2 * len(ops))]
    srv = Server(ops)
    srv.run(warm)
    srv.batches.clear()
    reqs = [Request(op=int(opi[i]), bdry=pools[opi[i]][0][rhs[i]], src=pools[opi[i]][1][rhs[i]],
                    t_arrival=float(ta[i])) for i in range(n_req)]
    srv.run(reqs)
    torch.cuda.synchronize()
    st = latency_stats(reqs)
    st.update({"rate_per_s": rate, "operators": len(ops), "resident_GB": resident / 1e9,
               "batches": len(srv.batches), "mean_batch": float(np.mean(srv.batches)), "precision": "fp64"})
    srv.free()
    for op in ops:
        op.free()
    return st


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run one plain device copy of 256 MiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design only)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_probe:
        n = 256 * 2 ** 20 // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8}), flush=True)
        return

    import paper_2503_17535_amd as hp
    import workloads as W

    dev = torch.device("cuda:0")
    t = hp.tree(2, DEPTH)
    sz = hp.sizes(t, P)
    pts = hp.leaf_points(t, P)
    bpts = hp.boundary_points(t, P)
    coeffs, bdry, src = W.helmholtz_inputs(pts, bpts, K_WAVE, NRHS)
    c_d = torch.tensor(coeffs, device=dev)
    b_d = torch.tensor(bdry, device=dev)
    s_d = torch.tensor(src, device=dev)
    u_d = torch.empty((NRHS, sz.n_leaves, sz.pts_per_leaf), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    flags = hp.FLAG_TIMING

    def step(record=None):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e2 = torch.cuda.Event(enable_timing=True)
        e0.record()
        op = hp.build(t, P, c_d, flags=flags)
        build_stages = op.stage_times()
        e1.record()
        op.solve(b_d, s_d, out=u_d)
        e2.record()
        solve_stages = op.stage_times()
        op.free()
        if record is not None:
            record.append((e0, e1, e2, build_stages + solve_stages))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    recs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(recs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    ms_step = wall * 1e3 / args.steps
    build_ms = float(np.mean([a.elapsed_time(b) for a, b, c, s in recs]))
    solve_ms = float(np.mean([b.elapsed_time(c) for a, b, c, s in recs]))
    stages = {}
    for *_, st in recs:
        for name, ms in st:
            stages.setdefault(name, []).append(ms)
    stages = {k: float(np.mean(v)) for k, v in stages.items()}

    # dominant kernel: the fused leaf factorization (one launch per build)
    leaf_ms = stages.get("leaf_factor", float("nan"))
    flops = leaf_flops(P) * sz.n_leaves
    achieved = flops / (leaf_ms * 1e-3) / 1e12
    roofline = {"kernel": "leaf2d_factor_kernel<16>", "bound": "alu", "achieved": achieved,
                "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                "traffic": measured_traffic(), "algorithmic_flops_per_launch": flops, "avg_launch_ms": leaf_ms}

    out = {
        "metric": METRIC,
        "value": sz.n_leaves * 1e3 / ms_step,
        "unit": "leaves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "2D Helmholtz k=40, q = 8 Gaussian bumps, depth-6 quadtree (4096 leaves), "
                               "p=16, build + 16-rhs solve", "n_leaves": sz.n_leaves, "p": P,
                   "depth": DEPTH, "nrhs": NRHS, "k": K_WAVE},
        "build_ms": build_ms, "solve_ms": solve_ms,
        "build_leaves_per_s": sz.n_leaves * 1e3 / build_ms,
        "solves_per_s": NRHS * 1e3 / solve_ms,
        "stages_ms": stages,
        "roofline": roofline,
    }
    out.update(solve_rates(hp, t, c_d, b_d, s_d, sz))
    out["refined"] = refined_solve(hp, t, c_d, b_d, s_d)
    if not args.no_serving:
        out["serving"] = serving(hp, W)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
