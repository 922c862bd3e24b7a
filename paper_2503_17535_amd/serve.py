"""Continuous-batching serving of solve requests against resident operators.

Each request names one resident operator and carries one right-hand side
(Dirichlet data and, optionally, a source; device tensors).  Requests arrive
over time (an open-loop stream replayed against the wall clock).

The operators are split into classes by the cost of one solve (by default by
tree depth: shallow, middle, deep), and every class has its own HIP stream,
batcher and in-flight queue.  The scheduler admits arrived requests of a
class while the class has a free in-flight slot, at most 16 right-hand sides
per operator and ``max_batch`` requests per batch are taken, and the bytes of
admitted, unfinished outputs stay within ``mem_budget``; each admitted set is
submitted as one batched solve on the class's stream.  Batches of different
classes therefore run at the same time on the device, and a request for a
shallow operator never waits behind the solve of a deep one; an operator is
only ever used on its class's stream, so the per-operator solve workspace is
reused in stream order.  Requests that arrive while a class's batch runs
join its next batch, which is submitted when the running one completes
(``max_inflight`` = 1: a second queued batch would only make them wait
longer).  At most four classes: the device runs four hardware queues per
process, and streams beyond that share a queue, which serializes them.

Precision: ``fp64`` submits one ``hps_solve_batch`` per batch (one launch per
pass stage over all operators of the class); ``fp32_refined`` solves the
requests of each operator in the batch together with the mixed-precision
solve (operators built with HPS_FLAG_FP32_COPY).

A request completes when the last kernel of its batch has finished on the
device: a timing event recorded after the batch on the class's stream, mapped
to the host clock through a reference event.  Latency = completion -
scheduled arrival.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

from . import FP32_REFINED, Batcher


@dataclasses.dataclass
class Request:
    op: int                      # index into the server's operators
    bdry: object                 # CUDA float64 [n_root_bdry]
    src: object = None           # CUDA float64 [n_leaves, p^2] or None
    t_arrival: float = 0.0       # scheduled arrival, seconds from the start of the run
    u: object = None             # output, allocated at admission
    t_admit: float = float("nan")
    t_done: float = float("nan")
    batch: int = -1


def depth_classes(ops, alone_from: int = 7):
    """Default classes: the operators of tree depth <= 5 together, those of
    depth 6 together, and every operator of depth >= alone_from in a class of
    its own (its solve reads gigabytes of stored operators; sharing a batch
    with another deep operator would double the time its requests wait)."""
    cls = collections.OrderedDict()
    for i, op in enumerate(ops):
        dep = op.tree.depth
        key = ("alone", i) if dep >= alone_from else min(max(dep, 5), alone_from - 1)
        cls.setdefault(key, []).append(i)
    return list(cls.values())


class _Class:
    def __init__(self, torch, members, stream):
        self.members = set(members)
        self.stream = stream
        self.batcher = Batcher()
        self.queue = collections.deque()
        self.inflight = collections.deque()      # ((start event, end event), requests, bytes)


class Server:
    def __init__(self, ops, max_rhs: int = 16, max_batch: int = 128, mem_budget: int = 64 << 30,
                 max_inflight: int = 1, classes=None, precision: str = "fp64"):
        import torch
        if precision not in ("fp64", "fp32_refined"):
            raise ValueError(precision)
        self.torch = torch
        self.ops = list(ops)
        self.max_rhs = max_rhs
        self.max_batch = max_batch
        self.mem_budget = mem_budget
        self.max_inflight = max_inflight
        self.precision = precision
        groups = classes if classes is not None else depth_classes(self.ops)
        if len(groups) > 4:
            raise ValueError("at most 4 operator classes (one stream each; the device has 4 hardware queues)")
        self.classes = [_Class(torch, g, torch.cuda.Stream()) for g in groups]
        self.class_of = {}
        for ci, g in enumerate(groups):
            for i in g:
                self.class_of[i] = ci
        if len(self.class_of) != len(self.ops):
            raise ValueError("every operator must belong to exactly one class")
        self.out_bytes = [op.sizes.n_leaves * op.sizes.pts_per_leaf * 8 for op in self.ops]
        self.batches = []            # number of requests per submitted batch
        self.trace = []              # (class, device start, device end) of every batch, seconds

    def _submit(self, cl, reqs, t_now):
        torch = self.torch
        per_op = collections.OrderedDict()
        for r in reqs:
            r.t_admit = t_now
            r.batch = len(self.batches)
            per_op.setdefault(r.op, []).append(r)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev0.record(cl.stream)
        with torch.cuda.stream(cl.stream):
            if self.precision == "fp64":
                items = []
                for k, rs in per_op.items():
                    s = self.ops[k].sizes
                    for r in rs:
                        r.u = torch.empty((s.n_leaves, s.pts_per_leaf), dtype=torch.float64, device=r.bdry.device)
                    src = [r.src for r in rs]
                    items.append((self.ops[k], [r.bdry for r in rs], None if all(x is None for x in src) else src,
                                  [r.u for r in rs]))
                cl.batcher.solve(items, stream=cl.stream)
            else:
                for k, rs in per_op.items():
                    op = self.ops[k]
                    bd = torch.stack([r.bdry for r in rs])
                    src = None
                    if any(r.src is not None for r in rs):
                        s = op.sizes
                        src = torch.stack([r.src if r.src is not None else
                                           torch.zeros((s.n_leaves, s.pts_per_leaf), dtype=torch.float64,
                                                       device=r.bdry.device) for r in rs])
                    u = op.solve(bd, src, stream=cl.stream, precision=FP32_REFINED)
                    for j, r in enumerate(rs):
                        r.u = u[j]
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(cl.stream)
        self.batches.append(len(reqs))
        return ev0, ev

    def run(self, requests, idle_sleep: float = 20e-6):
        """Replays ``requests`` (sorted by t_arrival) against the wall clock and
        returns them with t_admit / t_done filled in."""
        torch = self.torch
        pending = collections.deque(sorted(requests, key=lambda r: r.t_arrival))
        mem_used = 0
        done = 0
        n = len(pending)
        ref = torch.cuda.Event(enable_timing=True)
        ref.record()
        ref.synchronize()
        t0 = time.perf_counter()
        while done < n:
            now = time.perf_counter() - t0
            while pending and pending[0].t_arrival <= now:
                r = pending.popleft()
                self.classes[self.class_of[r.op]].queue.append(r)
            progressed = False
            for cl in self.classes:
                while cl.inflight and cl.inflight[0][0][1].query():
                    (ev0, ev), reqs, nbytes = cl.inflight.popleft()
                    t_done = ref.elapsed_time(ev) * 1e-3
                    self.trace.append((self.classes.index(cl), ref.elapsed_time(ev0) * 1e-3, t_done))
                    for r in reqs:
                        r.t_done = t_done
                    mem_used -= nbytes
                    done += len(reqs)
                if cl.queue and len(cl.inflight) < self.max_inflight:
                    count = collections.Counter()
                    admitted, rest, nbytes = [], collections.deque(), 0
                    for r in cl.queue:
                        b = self.out_bytes[r.op]
                        if (count[r.op] < self.max_rhs and len(admitted) < self.max_batch
                                and mem_used + nbytes + b <= self.mem_budget):
                            count[r.op] += 1
                            admitted.append(r)
                            nbytes += b
                        else:
                            rest.append(r)
                    if admitted:
                        cl.queue = rest
                        ev = self._submit(cl, admitted, now)
                        cl.inflight.append((ev, admitted, nbytes))
                        mem_used += nbytes
                        progressed = True
            if not progressed and not (pending and pending[0].t_arrival <= time.perf_counter() - t0):
                time.sleep(idle_sleep)
        return requests

    def free(self):
        self.torch.cuda.synchronize()
        for cl in self.classes:
            cl.batcher.free()


def latency_stats(requests):
    lat = np.array([r.t_done - r.t_arrival for r in requests]) * 1e3
    t_first = min(r.t_arrival for r in requests)
    t_last = max(r.t_done for r in requests)
    return {"requests": len(requests), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
            "max_ms": float(lat.max()), "solves_per_s": len(requests) / (t_last - t_first)}
