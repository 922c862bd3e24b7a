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

Beside the headline line: the roofline of the leaf kernel (dominant), of the
solve (HBM) and per merge level (FP64); the mixed-precision solve; the small
2D Poisson latency, the 3D div-grad build/solve with its peak device memory,
the 32-field misfit gradient, continuous-batching serving; and the CPU oracle
on the full workload, whose solution gives every GPU path's error.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
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


def merge_levels_2d(depth: int, p: int):
    """(level, nodes, m, flops) of the 2D merges: the explicit inverse of D
    (2 m^3), S = -D^{-1} C (2 m^3: C's zero blocks skipped) and, below the
    root, T = A + B S (4 m^3: B's zero blocks skipped).  The accuracy guard's
    Newton-Schulz steps are extra work and not counted."""
    q = p - 2
    out = []
    for lev in range(depth - 1, -1, -1):
        nodes = 4 ** lev
        m = 4 * q * 2 ** (depth - 1 - lev)
        per = 2.0 * m ** 3 + 2.0 * m ** 3 + (4.0 * m ** 3 if lev > 0 else 0.0)
        out.append((lev, nodes, m, nodes * per))
    return out


def solve_bytes_2d(depth: int, p: int, nrhs: int, with_src: bool = True) -> float:
    """Algorithmic HBM bytes of one solve pass over nrhs right-hand sides:
    every stored operator read once (leaf LU factors when a source is given,
    Y_int; per merge D^{-1}, S and the nonzero blocks of B), the source read
    and the solution written."""
    q = p - 2
    nl, ni, nb, npts = 4 ** depth, q * q, 4 * q, p * p
    b = nl * ni * nb * 8.0 + (nl * ni * ni * 8.0 if with_src else 0.0)
    for lev, nodes, m, _ in merge_levels_2d(depth, p):
        b += nodes * (m * m + m * 2 * m + m * m) * 8.0     # Z, S (m x 2m), 4 blocks (m/2)^2 of B
    b += nrhs * nl * npts * 8.0 * (2 if with_src else 1)
    return b


def host_info():
    info = {"os_cpu_count": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)),
            "machine": platform.machine()}
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in txt.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "CPU(s)", "Thread(s) per core", "Socket(s)"):
                info[k.strip()] = v.strip()
    except Exception:  # pragma: no cover
        pass
    return info


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        return os.cpu_count() or 1


def cpu_baseline(coeffs, bdry, src):
    """The oracle (plain NumPy/SciPy, LAPACK on the host's cores) on the full
    workload: build + 16 solves, once.  Returns the record and the oracle's
    solution (every GPU path's error is taken against it).  A 256-leaf
    subtree is timed with all threads and with one beside it."""
    import numpy as np
    import workloads as W
    from oracle import hps as ohps
    tree = ohps.Tree(2, DEPTH)
    t0 = time.perf_counter()
    op = ohps.build(tree, P, coeffs)
    t1 = time.perf_counter()
    ref = np.stack([ohps.solve(op, bdry[r], src[r]) for r in range(NRHS)])
    t2 = time.perf_counter()
    del op
    nl = tree.n_leaves
    rec = {"value": nl / (t2 - t0), "unit": "leaves/s", "cores": int(blas_threads()), "kind": "oracle",
           "sample": f"the full workload once: oracle build of all {nl} leaves (p={P}, k={K_WAVE:g}) + {NRHS} "
                     f"solves; build {t1 - t0:.2f}s, solves {t2 - t1:.2f}s",
           "build_leaves_per_s": nl / (t1 - t0), "solves_per_s": NRHS / (t2 - t1), "host": host_info()}
    try:
        # the same 256-leaf quadrant subtree (depth 4, same inputs) with all
        # threads and with one, so that the two figures compare like with like
        from threadpoolctl import threadpool_limits
        sub = ohps.Tree(2, 4, -1.0, -0.5)
        disc = ohps.LeafDisc(2, P)
        pts = sub.leaf_points(disc)
        c1, b1, s1 = W.helmholtz_inputs(pts, sub.root_boundary_points(disc), K_WAVE, 1)

        def timed():
            t0 = time.perf_counter()
            o1 = ohps.build(sub, P, c1)
            t1 = time.perf_counter()
            ohps.solve(o1, b1[0], s1[0])
            return sub.n_leaves / (t1 - t0), time.perf_counter() - t1
        all_b, all_s = timed()
        with threadpool_limits(1):
            one_b, one_s = timed()
        rec["subtree"] = {"sample": f"build of a {sub.n_leaves}-leaf subtree (depth 4) + 1 solve",
                          "threads": int(blas_threads()), "build_leaves_per_s": all_b, "solve_s": all_s,
                          "one_thread_build_leaves_per_s": one_b, "one_thread_solve_s": one_s}
    except Exception as e:  # pragma: no cover
        rec["subtree"] = {"error": str(e)}
    return rec, ref


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


def rel_err(u, ref):
    import numpy as np
    return float(max(np.abs(u[r] - ref[r]).max() / np.abs(ref[r]).max() for r in range(ref.shape[0])))


def solve_rates(hp, t, c_d, b_d, s_d):
    """Solve-only rates of one resident operator: 16 and 1 right-hand sides
    (median of 5 after a warm-up), and the solve's HBM roofline."""
    op = hp.build(t, P, c_d)
    u16 = op.solve(b_d, s_d)
    ms16 = _median_ms(lambda: op.solve(b_d, s_d, out=u16))
    b1, s1 = b_d[:1].contiguous(), s_d[:1].contiguous()
    u1 = op.solve(b1, s1)
    ms1 = _median_ms(lambda: op.solve(b1, s1, out=u1))
    op.free()
    by = solve_bytes_2d(DEPTH, P, NRHS)
    gbs = by / (ms16 * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS,
            "algorithmic_bytes": by, "ms": ms16}
    return {"solve16_ms": ms16, "solves_per_s_nrhs16": NRHS * 1e3 / ms16,
            "solve1_ms": ms1, "solves_per_s_nrhs1": 1e3 / ms1}, roof, u16


def refined_solve(hp, t, c_d, b_d, s_d):
    """Mixed-precision solve of the same workload (fp32 operator copies, fp64
    residual refinement)."""
    import torch
    op = hp.build(t, P, c_d, flags=hp.FLAG_FP32_COPY)
    u64 = op.solve(b_d, s_d)
    sweeps = op.refine_sweeps()
    u = op.solve(b_d, s_d, precision=hp.FP32_REFINED)
    ms = _median_ms(lambda: op.solve(b_d, s_d, out=u, precision=hp.FP32_REFINED))
    diff = ((u - u64).abs().amax(dim=(1, 2)) / u64.abs().amax(dim=(1, 2))).max().item()
    op.free()
    # capacity: fp64 operators freed once the fp32 copies exist
    op64 = hp.build(t, P, c_d)
    op32 = hp.build(t, P, c_d, flags=hp.FLAG_FP32_ONLY)
    u32 = op32.solve(b_d, s_d, precision=hp.FP32_REFINED)
    same = bool(torch.equal(u32, u))
    res64, res32 = op64.nbytes, op32.nbytes
    op64.free()
    op32.free()
    torch.cuda.synchronize()
    return {"sweeps": sweeps, "solve16_ms": ms, "solves_per_s": NRHS * 1e3 / ms,
            "max_rel_diff_to_fp64": diff, "resident_GB_fp64": res64 / 1e9, "resident_GB_fp32_only": res32 / 1e9,
            "fp32_only_equals_refined": same}, u


def poisson_latency(hp, W):
    """Small 2D Poisson: -Lap u = 2 pi^2 sin(pi x) sin(pi y), depth 2 (16
    leaves), p = 8: build + 1 solve latency (too small for either roofline)."""
    import numpy as np
    import torch
    t = hp.tree(2, 2)
    pts = hp.leaf_points(t, 8)
    bpts = hp.boundary_points(t, 8)
    c = torch.tensor(W.coeffs_poisson(pts), device="cuda:0")
    g = torch.tensor(W.sinsin(bpts)[None], device="cuda:0")
    f = torch.tensor(W.sinsin_minus_laplacian(pts)[None], device="cuda:0")
    u = torch.empty((1, 16, 64), dtype=torch.float64, device="cuda:0")

    def once():
        op = hp.build(t, 8, c)
        op.solve(g, f, out=u)
        op.free()
    for _ in range(3):
        once()
    torch.cuda.synchronize()
    wall = []
    for _ in range(50):
        t0 = time.perf_counter()
        once()
        torch.cuda.synchronize()
        wall.append((time.perf_counter() - t0) * 1e3)
    err = float(np.abs(u[0].cpu().numpy() - W.sinsin(pts)).max())
    return {"workload": "2D Poisson depth 2 (16 leaves), p=8, sin(pi x) sin(pi y)",
            "build_solve_latency_ms_p50": float(np.median(wall)), "p99_ms": float(np.percentile(wall, 99)),
            "abs_err_vs_exact": err}


def divgrad_3d(hp, W):
    """3D variable-coefficient Poisson div(a grad u) = f, a = 1 + 0.5 sin
    product, octree depth 3 (512 leaves), p = 12, 10x10 Gauss face nodes;
    manufactured u = sin sin sin + xyz.  Build and one solve, device times,
    and the library's peak device memory over build + solve."""
    import numpy as np
    import torch
    p, L = 12, 3
    t = hp.tree(3, L)
    pts = hp.leaf_points(t, p)
    bpts = hp.boundary_points(t, p)
    prm = W.draw_sinprod(W.rng(3, 0))
    c = torch.tensor(W.coeffs_divgrad(pts, prm), device="cuda:0")
    a, ga = W.eval_sinprod(prm, pts)
    ue, gu, lap = W.sin3_plus_xyz(pts)
    g = torch.tensor(W.sin3_plus_xyz(bpts)[0][None], device="cuda:0")
    f = torch.tensor((a * lap + np.sum(ga * gu, axis=-1))[None], device="cuda:0")
    torch.cuda.synchronize()
    base, _ = hp.mem_stats(reset_peak=True)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    op = hp.build(t, p, c)
    e[1].record()
    u = op.solve(g, f)
    e[2].record()
    e[2].synchronize()
    _, peak = hp.mem_stats()
    resident = op.nbytes
    ms_solve = _median_ms(lambda: op.solve(g, f, out=u), reps=3)
    op.free()
    err = float(np.abs(u[0].cpu().numpy() - ue).max() / np.abs(ue).max())
    return {"workload": "3D div(a grad u) = f, octree depth 3 (512 leaves), p=12, root D 19200",
            "build_ms": e[0].elapsed_time(e[1]), "solve_ms": ms_solve, "first_solve_ms": e[1].elapsed_time(e[2]),
            "build_leaves_per_s": 512 * 1e3 / e[0].elapsed_time(e[1]),
            "peak_device_GB": (peak - base) / 1e9, "resident_GB": resident / 1e9,
            "rel_err_vs_manufactured": err}


def subtree_recomputation(hp, W, deep: bool = False):
    """2D p = 16 trees of depth 8 and 9 (16.8M and 67.1M unknowns), the sizes
    of the paper's subtree-recomputation runs: build + one solve with a
    source (local solves, merges, downward pass: what the paper times) of the
    resident operator and of the recomputing one (hps_build_subtrees with
    5- and 6-level subtrees), the library's peak device memory of each, and
    the error against the problem's exact polynomial solution.  With deep,
    also depth 10 (268M unknowns, 7-level subtrees), whose resident operator
    (679 GB) does not fit one GPU: recomputation only."""
    import numpy as np
    import torch
    out = []
    for L, sd in ((8, 5), (9, 6)) + (((10, 7),) if deep else ()):
        p = 16
        t = hp.tree(2, L)
        pts = hp.leaf_points(t, p)
        bpts = hp.boundary_points(t, p)
        c, f, g, uex = W.poly5_problem(pts, bpts)
        del pts
        ct = torch.tensor(c, device="cuda:0")
        del c
        ft = torch.tensor(f[None], device="cuda:0")
        gt = torch.tensor(g[None], device="cuda:0")
        u = torch.empty_like(ft)
        scale = np.abs(uex).max()
        rec = {"depth": L, "p": p, "unknowns": int(4 ** L * p * p), "subtree_depth": sd,
               "resident_operator_GB": hp.footprint(t, p) / 1e9}
        fits = rec["resident_operator_GB"] < 250.0
        if not fits:
            rec["resident"] = {"skipped": "resident operator larger than the GPU's memory"}
        for mode in (("resident", "recompute") if fits else ("recompute",)):
            torch.cuda.synchronize()
            base, _ = hp.mem_stats(reset_peak=True)
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record()
            op = hp.build_subtrees(t, p, ct, sd) if mode == "recompute" else hp.build(t, p, ct)
            e[1].record()
            op.solve(gt, ft, out=u)
            e[2].record()
            e[2].synchronize()
            _, peak = hp.mem_stats()
            op.free()
            rec[mode] = {"build_s": e[0].elapsed_time(e[1]) * 1e-3, "solve_s": e[1].elapsed_time(e[2]) * 1e-3,
                         "total_s": e[0].elapsed_time(e[2]) * 1e-3, "peak_device_GB": (peak - base) / 1e9,
                         "rel_err_vs_exact": float(np.abs(u[0].cpu().numpy() - uex).max() / scale)}
        out.append(rec)
        del ct, ft, gt, u
        torch.cuda.empty_cache()
    return {"workload": "2D variable-coefficient problem with a degree-5 polynomial solution, p=16",
            "runs": out}


def iti_helmholtz(hp, W):
    """The ItI variant (hps_build_iti) on the paper's ItI problem (Section
    5.1: Laplace u + (1 + e^{-50|x|^2}) u = f, u_n + i u = g, u = e^{20ix} +
    e^{30iy}), p = 16, depths 5 and 6: build and one solve (device times),
    resident bytes and the error against the exact solution at the interior
    points."""
    import numpy as np
    import torch
    out = []
    p = 16
    for L in (5, 6):
        t = hp.tree(2, L)
        pts = hp.leaf_points(t, p)
        bpts = hp.boundary_points(t, p)
        c, f, g, uex = W.iti_problem(pts, bpts)
        ct = torch.tensor(c, device="cuda:0")
        ft = torch.tensor(f[None], device="cuda:0")
        gt = torch.tensor(g[None], device="cuda:0")
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        torch.cuda.synchronize()
        e[0].record()
        op = hp.build_iti(t, p, ct, 1.0)
        e[1].record()
        u = op.solve(gt, ft)
        e[2].record()
        e[2].synchronize()
        ms_solve = _median_ms(lambda: op.solve(gt, ft, out=u), reps=3)
        resident = op.nbytes
        op.free()
        q = (np.arange(p * p) % p > 0) & (np.arange(p * p) % p < p - 1) & \
            (np.arange(p * p) // p > 0) & (np.arange(p * p) // p < p - 1)
        uu = u[0].cpu().numpy()[:, q]
        err = float(np.abs(uu - uex[:, q]).max() / np.abs(uex[:, q]).max())
        out.append({"depth": L, "p": p, "unknowns": int(4 ** L * p * p), "build_ms": e[0].elapsed_time(e[1]),
                    "solve_ms": ms_solve, "first_solve_ms": e[1].elapsed_time(e[2]),
                    "resident_GB": resident / 1e9, "rel_err_vs_exact": err})
        del ct, ft, gt, u
        torch.cuda.empty_cache()
    return {"workload": "ItI variant, paper's ItI problem (eta = 1), p=16", "runs": out}


def adaptive_3d(hp, W):
    """Section 4.2 on the paper's wavefront problem (Poisson on [0, 1]^3,
    u = arctan(10 |x - c| - 0.7), centre off the dyadic grid): the adaptive
    tree (criterion on the GPU), its build (the second one, with the device
    memory cache warm; host planning included) and solve (device times), root
    D, peak device memory and error against the exact u, beside the uniform
    tree of the same finest level where it fits (Section 4.2's table)."""
    import time

    import numpy as np
    import torch
    dev = "cuda:0"
    funcs = [lambda x: W.wavefront_u(x), lambda x: W.wavefront_f(x)]

    def run(build, pts, bpts):
        c = torch.tensor(W.coeffs_poisson(pts), device=dev)
        g = torch.tensor(W.wavefront_u(bpts)[None], device=dev)
        f = torch.tensor(W.wavefront_f(pts)[None], device=dev)
        build(c).free()  # warm the library's device memory cache
        torch.cuda.synchronize()
        base, _ = hp.mem_stats(reset_peak=True)
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        e[0].record()
        op = build(c)
        e[1].record()
        e[1].synchronize()
        u = op.solve(g, f)
        torch.cuda.synchronize()
        _, peak = hp.mem_stats()
        ms_solve = _median_ms(lambda: op.solve(g, f, out=u), reps=3)
        ue = W.wavefront_u(pts)
        err = float(np.abs(u[0].cpu().numpy() - ue).max() / np.abs(ue).max())
        rec = {"build_ms": e[0].elapsed_time(e[1]), "solve_ms": ms_solve, "peak_device_GB": (peak - base) / 1e9,
               "resident_GB": op.nbytes / 1e9, "rel_err_vs_exact": err}
        op.free()
        return rec

    out = []
    for p, eps, cap in ((8, 1e-4, 4), (10, 1e-5, 3), (12, 1e-5, 3)):
        t0 = time.perf_counter()
        t = hp.adaptive_tree(funcs, p, eps, cap)
        tree_s = time.perf_counter() - t0
        pts, bpts = t.points(p, 0), t.points(p, 2)
        box = {}

        def build_a(c, t=t, p=p, box=box):
            op = hp.build_adaptive(t, p, c)
            box["D"] = op.root_D
            return op

        ra = run(build_a, pts, bpts)
        ra.update({"leaves": t.n_leaves, "levels": sorted({int(x) for x in t.leaves[:, 0]}), "root_D": box["D"],
                   "tree_s": tree_s})
        L = int(t.leaves[:, 0].max())
        tu = hp.tree(3, L, 0.0, 1.0)
        su = hp.sizes(tu, p)
        ru = {"leaves": int(su.n_leaves), "root_D": int(su.root_D)}
        try:
            ru.update(run(lambda c, tu=tu, p=p: hp.build(tu, p, c), hp.leaf_points(tu, p), hp.boundary_points(tu, p)))
        except hp.HPSError as e:  # e.g. the root Schur complement beyond the Gauss-Jordan limit
            ru["skipped"] = str(e)
        out.append({"p": p, "eps": eps, "max_level": cap, "adaptive": ra, "uniform": ru})
        torch.cuda.empty_cache()
    return {"workload": "adaptive 3D, paper's wavefront problem (Poisson, u = arctan(10 r - 0.7))", "runs": out}


def misfit_gradients(hp, W, with_oracle: bool):
    """Misfit gradient workload: J(q) = ||E u(q) - u_obs||^2 at 256 points,
    2D Helmholtz k = 20, depth 5, p = 16, 32 seeded fields q: per field a
    build, a solve, the adjoint solve and the coefficient gradient (through
    torch.autograd).  Time for all 32, and the error of field 0's gradient
    against the oracle's adjoint gradient."""
    import numpy as np
    import torch
    from paper_2503_17535_amd.autograd import solve as hsolve
    d, p, L = 2, 16, 5
    dev = torch.device("cuda:0")
    t = hp.tree(d, L)
    pts = hp.leaf_points(t, p)
    bpts = hp.boundary_points(t, p)
    inp = W.differentiation_inputs(pts, bpts)
    k = inp["k"]
    bd = torch.tensor(inp["bdry"], device=dev)
    src = torch.tensor(inp["src"], device=dev)
    leaf, wts = hp.interp_weights(t, p, inp["x_obs"])
    leaf_t, wts_t = torch.tensor(leaf, device=dev), torch.tensor(wts, device=dev)

    def coeffs(q):
        nl, npts = q.shape
        c = torch.zeros((nl, 5, npts), dtype=torch.float64, device=dev)
        c[:, 0] = -1.0
        c[:, 2] = -1.0
        return torch.cat([c, (-(k * k) * (1.0 + q))[:, None]], dim=1)

    def observe(u):
        return (wts_t * u[0, leaf_t, :]).sum(-1)

    with torch.no_grad():
        u_obs = observe(hsolve(t, p, coeffs(torch.tensor(inp["q_star"], device=dev)), bd, src))
    qs = [torch.tensor(inp["q"][f], device=dev, requires_grad=True) for f in range(inp["q"].shape[0])]

    def run():
        grads = []
        for q in qs:
            q.grad = None
            u = hsolve(t, p, coeffs(q), bd, src)
            ((observe(u) - u_obs) ** 2).sum().backward()
            grads.append(q.grad)
        return grads
    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    grads = run()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rec = {"workload": "misfit gradient, 2D Helmholtz k=20, depth 5 (1024 leaves), p=16, 256 points, 32 fields",
           "fields": len(qs), "total_ms": wall * 1e3, "ms_per_field": wall * 1e3 / len(qs),
           "gradients_per_s": len(qs) / wall}
    if with_oracle:
        from oracle import adjoint as A
        from oracle import hps as ohps
        tree = ohps.Tree(d, L)
        disc = ohps.LeafDisc(d, p)
        opts = tree.leaf_points(disc)
        op_s = ohps.build(tree, p, W.coeffs_helmholtz(opts, k, inp["q_star"]))
        oleaf, oW = A.observation(tree, p, inp["x_obs"])
        uo_obs = np.einsum("mk,mk->m", oW, ohps.solve(op_s, inp["bdry"][0], inp["src"][0])[oleaf])
        del op_s
        op0 = ohps.build(tree, p, W.coeffs_helmholtz(opts, k, inp["q"][0]))
        u0 = ohps.solve(op0, inp["bdry"][0], inp["src"][0])
        lam0, _ = A.hps_adjoint(op0, A.misfit_weight(u0, oleaf, oW, uo_obs))
        ref = -(k * k) * A.coeff_grad(tree, p, u0[None], lam0[None])[:, 5]
        g0 = grads[0].cpu().numpy()
        rec["field0_rel_err_vs_oracle"] = float(np.abs(g0 - ref).max() / np.abs(ref).max())
    return rec


def serving(hp, W, n_req=4096, rate=2000.0):
    """Continuous-batching serving (see paper_2503_17535_amd.serve): 8
    resident Helmholtz operators (depths 4-7, p 12/16, k 10-40, built with
    fp32 copies so both precisions run on them), 4096 requests with
    exponential inter-arrival times at 2000/s replayed against the wall clock,
    each for a uniformly chosen operator with its own seeded Fourier boundary
    data and source bump (generated on the device before the run).  Latency =
    device completion - scheduled arrival.  Runs: fp64 and fp32+fp64
    refinement at 2000/s, and an fp64 rate sweep on the first 1024 requests."""
    import numpy as np
    import torch
    from paper_2503_17535_amd.serve import Request, Server, latency_stats
    dev = torch.device("cuda:0")
    ops, pts_d, four = [], [], []
    for k, (L, p, kw) in enumerate(W.SERVING_OPS):
        tt = hp.tree(2, L)
        pts = hp.leaf_points(tt, p)
        bpts = hp.boundary_points(tt, p)
        c, _, _ = W.helmholtz_inputs(pts, bpts, kw, 1, config=4, op_seed=k)
        ops.append(hp.build(tt, p, torch.tensor(c, device=dev), flags=hp.FLAG_FP32_COPY))
        pts_d.append(torch.tensor(pts, device=dev))
        # Fourier basis in perimeter arclength at this operator's boundary points
        sarc = W.perimeter_arclength(bpts)
        m = np.arange(17)[:, None]
        four.append((torch.tensor(np.cos(2 * np.pi * m * sarc / 8.0), device=dev),
                     torch.tensor(np.sin(2 * np.pi * m * sarc / 8.0), device=dev)))
    resident = sum(op.nbytes for op in ops)
    ta, opi, _ = W.serving_arrivals(n_req, rate, len(ops), 1)
    data = []
    for i in range(n_req):
        fo, sb = W.serving_request_params(i)
        k = int(opi[i])
        cb, sn = four[k]
        bd = torch.tensor(fo["a"], device=dev) @ cb + torch.tensor(fo["b"], device=dev) @ sn
        z = torch.tensor(sb["centres"][0], device=dev)
        src = float(sb["amps"][0]) * torch.exp(-((pts_d[k] - z) ** 2).sum(-1) / (2 * 0.1 ** 2))
        data.append((bd, src))
    torch.cuda.synchronize()
    solo = []
    for op in ops:      # one-rhs solve of each operator alone (median of 5)
        k = ops.index(op)
        i = int(np.nonzero(opi == k)[0][0])
        b1, s1 = data[i][0][None].contiguous(), data[i][1][None].contiguous()
        u1 = op.solve(b1, s1)
        solo.append(_median_ms(lambda: op.solve(b1, s1, out=u1)))

    def run(prec, r, n):
        t_a, o_i, _ = W.serving_arrivals(n_req, r, len(ops), 1)
        srv = Server(ops, precision=prec)
        warm = [Request(op=k, bdry=data[int(np.nonzero(opi == k)[0][0])][0],
                        src=data[int(np.nonzero(opi == k)[0][0])][1], t_arrival=0.0) for k in range(len(ops))]
        srv.run(warm)
        srv.batches.clear()
        reqs = [Request(op=int(o_i[i]), bdry=data[i][0], src=data[i][1], t_arrival=float(t_a[i]))
                for i in range(n)]
        srv.run(reqs)
        torch.cuda.synchronize()
        st = latency_stats(reqs)
        st.update({"rate_per_s": r, "batches": len(srv.batches), "mean_batch": float(np.mean(srv.batches)),
                   "precision": prec})
        srv.free()
        return st, reqs

    fp64, reqs64 = run("fp64", rate, n_req)
    ref32, reqs32 = run("fp32_refined", rate, n_req)
    # largest relative difference of a refined result to the fp64 result of
    # the same request (both are checked against the oracle in the tests)
    diff = max(((a.u - b.u).abs().max() / b.u.abs().max()).item() for a, b in zip(reqs32[::64], reqs64[::64]))
    ref32["max_rel_diff_to_fp64"] = diff
    del reqs64, reqs32
    sweep = [run("fp64", r, 1024)[0] for r in (1000.0, 4000.0, 8000.0)]
    out = dict(fp64)
    out.update({"operators": len(ops), "resident_GB": resident / 1e9, "classes": "depth <= 5 | 6 | 7",
                "solo_1rhs_ms": solo, "p99_over_deepest_solo": fp64["p99_ms"] / max(solo),
                "fp32_refined": ref32, "rate_sweep_fp64": sweep})
    for op in ops:
        op.free()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--deep", action="store_true",
                    help="add the depth-10 (268M unknowns) subtree-recomputation run (about 2 minutes, most of it "
                         "generating its inputs on the host)")
    ap.add_argument("--no-extra", action="store_true",
                    help="only the headline workload (no 2D Poisson, 3D, misfit-gradient or recomputation legs)")
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

    def step():
        # one step: build and first 16-rhs solve in one call (hps_build_solve:
        # the sources' leaf solves run beside the top merge levels), then free
        op, _ = hp.build_solve(t, P, c_d, b_d, s_d, out=u_d)
        op.free()

    def split_step(record):
        # the same work as separate build and solve calls with per-stage device
        # times (HPS_FLAG_TIMING): the build / solve split and the stage table
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
        record.append((e0, e1, e2, build_stages + solve_stages))

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    recs = []
    for _ in range(max(2, min(args.steps, 5))):
        split_step(recs)
    torch.cuda.synchronize()

    ms_step = wall * 1e3 / args.steps
    build_ms = float(np.mean([a.elapsed_time(b) for a, b, c, s in recs]))
    solve_ms = float(np.mean([b.elapsed_time(c) for a, b, c, s in recs]))
    # per step: device time of every stage summed over its launches (a
    # quadrant-pipelined build records the leaf factorization as four launches
    # and every merge level below the root as four shares)
    stages, counts = {}, {}
    for *_, st in recs:
        per, cnt = {}, {}
        for name, ms in st:
            per[name] = per.get(name, 0.0) + ms
            cnt[name] = cnt.get(name, 0) + 1
        for name in per:
            stages.setdefault(name, []).append(per[name])
            counts[name] = cnt[name]
    stages = {k: float(np.mean(v)) for k, v in stages.items()}

    # dominant kernel: the fused leaf factorization
    n_leaf_launches = counts.get("leaf_factor", 1)
    leaf_ms = stages.get("leaf_factor", float("nan")) / n_leaf_launches
    flops = leaf_flops(P) * sz.n_leaves / n_leaf_launches
    achieved = flops / (leaf_ms * 1e-3) / 1e12
    roofline = {"kernel": "leaf2d_factor_kernel<16>", "bound": "alu", "achieved": achieved,
                "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                "traffic": measured_traffic(), "algorithmic_flops_per_launch": flops, "avg_launch_ms": leaf_ms,
                "launches_per_build": n_leaf_launches}
    merge_roof = []
    for lev, nodes, m, fl in merge_levels_2d(DEPTH, P):
        ms = stages.get(f"merge_l{lev}", float("nan"))
        tf = fl / (ms * 1e-3) / 1e12
        merge_roof.append({"level": lev, "nodes": nodes, "m": m, "gflop": fl / 1e9, "ms": ms, "tflops": tf,
                           "frac": tf / PEAK_FP64_TFLOPS})

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
        "step_call": "hps_build_solve (build + first solve, sources' leaf part on a second stream)",
        "build_ms": build_ms, "solve_ms": solve_ms,
        "separate_calls_ms": build_ms + solve_ms,
        "build_leaves_per_s": sz.n_leaves * 1e3 / build_ms,
        "solves_per_s": NRHS * 1e3 / solve_ms,
        "stages_ms": stages,
        "roofline": roofline,
        "roofline_merge_levels": merge_roof,
    }
    rates, roof_solve, u64 = solve_rates(hp, t, c_d, b_d, s_d)
    out.update(rates)
    out["roofline_solve"] = roof_solve
    out["refined"], u_ref32 = refined_solve(hp, t, c_d, b_d, s_d)
    if not args.no_extra:
        out["poisson2d_latency"] = poisson_latency(hp, W)
        out["divgrad3d"] = divgrad_3d(hp, W)
        out["misfit_gradient"] = misfit_gradients(hp, W, with_oracle=not args.no_cpu_baseline)
        out["subtree_recomputation"] = subtree_recomputation(hp, W, deep=args.deep)
        out["iti"] = iti_helmholtz(hp, W)
        out["adaptive3d"] = adaptive_3d(hp, W)
    if not args.no_serving:
        out["serving"] = serving(hp, W)
    if not args.no_cpu_baseline:
        rec, ref = cpu_baseline(coeffs, bdry, src)
        out["cpu_baseline"] = rec
        out["rel_err_vs_oracle"] = {"fp64_step": rel_err(u_d.cpu().numpy(), ref),
                                    "fp64_solve": rel_err(u64.cpu().numpy(), ref),
                                    "fp32_refined": rel_err(u_ref32.cpu().numpy(), ref)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
