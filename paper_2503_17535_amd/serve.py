"""Continuous-batching serving of solve requests against resident operators.

Each request names one resident operator and carries one right-hand side
(Dirichlet data and, optionally, a source; device tensors).  Requests arrive
over time (an open-loop stream replayed against the wall clock).  The
scheduler admits arrived requests while there are free slots (at most 16
right-hand sides per operator and ``max_batch`` requests per batch) and free
output memory (the bytes of admitted, unfinished outputs stay within
``mem_budget``), and submits each admitted set as one batched solve: one
launch per pass stage over all operators and right-hand sides
(``hps_solve_batch``).  Up to ``max_inflight`` batches are queued on the
device, so requests that arrive while a batch runs join the next one without
waiting for the first to finish.

A request completes when the last kernel of its batch has finished on the
device: a timing event recorded after the batch, mapped to the host clock
through a reference event.  Latency = completion - scheduled arrival.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

from . import Batcher


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


class Server:
    def __init__(self, ops, max_rhs: int = 16, max_batch: int = 128, mem_budget: int = 8 << 30,
                 max_inflight: int = 2, stream=None):
        import torch
        self.torch = torch
        self.ops = list(ops)
        self.max_rhs = max_rhs
        self.max_batch = max_batch
        self.mem_budget = mem_budget
        self.max_inflight = max_inflight
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.batcher = Batcher()
        self.out_bytes = [op.sizes.n_leaves * op.sizes.pts_per_leaf * 8 for op in self.ops]
        self.batches = []            # number of requests per submitted batch

    def _submit(self, reqs, t_now):
        torch = self.torch
        per_op = collections.OrderedDict()
        for r in reqs:
            s = self.ops[r.op].sizes
            r.u = torch.empty((s.n_leaves, s.pts_per_leaf), dtype=torch.float64, device=r.bdry.device)
            r.t_admit = t_now
            r.batch = len(self.batches)
            per_op.setdefault(r.op, []).append(r)
        items = []
        for k, rs in per_op.items():
            src = [r.src for r in rs]
            items.append((self.ops[k], [r.bdry for r in rs], None if all(x is None for x in src) else src,
                          [r.u for r in rs]))
        self.batcher.solve(items, stream=self.stream)
        ev = torch.cuda.Event(enable_timing=True)
        ev.record(self.stream)
        self.batches.append(len(reqs))
        return ev

    def run(self, requests, idle_sleep: float = 20e-6):
        """Replays ``requests`` (sorted by t_arrival) against the wall clock and
        returns them with t_admit / t_done filled in."""
        torch = self.torch
        pending = collections.deque(sorted(requests, key=lambda r: r.t_arrival))
        queue = collections.deque()
        inflight = collections.deque()     # (event, requests, bytes)
        mem_used = 0
        done = 0
        n = len(pending)
        ref = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(self.stream):
            ref.record(self.stream)
            ref.synchronize()
            t0 = time.perf_counter()
            while done < n:
                now = time.perf_counter() - t0
                while pending and pending[0].t_arrival <= now:
                    queue.append(pending.popleft())
                while inflight and inflight[0][0].query():
                    ev, reqs, nbytes = inflight.popleft()
                    t_done = ref.elapsed_time(ev) * 1e-3
                    for r in reqs:
                        r.t_done = t_done
                    mem_used -= nbytes
                    done += len(reqs)
                if queue and len(inflight) < self.max_inflight:
                    count = collections.Counter()
                    admitted, rest, nbytes = [], collections.deque(), 0
                    for r in queue:
                        b = self.out_bytes[r.op]
                        if (count[r.op] < self.max_rhs and len(admitted) < self.max_batch
                                and mem_used + nbytes + b <= self.mem_budget):
                            count[r.op] += 1
                            admitted.append(r)
                            nbytes += b
                        else:
                            rest.append(r)
                    if admitted:
                        queue = rest
                        ev = self._submit(admitted, now)
                        inflight.append((ev, admitted, nbytes))
                        mem_used += nbytes
                        continue
                if not (pending and pending[0].t_arrival <= time.perf_counter() - t0):
                    time.sleep(idle_sleep)
        return requests

    def free(self):
        self.batcher.free()


def latency_stats(requests):
    lat = np.array([r.t_done - r.t_arrival for r in requests]) * 1e3
    t_first = min(r.t_arrival for r in requests)
    t_last = max(r.t_done for r in requests)
    return {"requests": len(requests), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
            "max_ms": float(lat.max()), "solves_per_s": len(requests) / (t_last - t_first)}
