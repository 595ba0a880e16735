"""Serving loop for motif-counting requests on resident graphs.

Requests name a graph of a loaded batch (pg_batch_load); the loop admits
them as they arrive into asynchronous slots (pg_batch_slot_*), each slot on
its own stream, so work admitted while other work runs overlaps with it on
the device (continuous batching).  Admission is bounded by a device-memory
footprint budget: a request holds its graph's CSR bytes plus its output
row until it completes.  Every request's latency is completion minus
arrival on the host wall clock.

All mining runs in the HIP library; this module only schedules.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import binding


@dataclass
class ServeStats:
    n_requests: int
    elapsed_s: float
    throughput: float            # completed requests per second
    p50_ms: float
    p99_ms: float
    mean_batch: float
    max_inflight_bytes: int
    latencies_ms: np.ndarray = field(repr=False)
    results: np.ndarray = field(repr=False)   # rows in request order


def graph_footprints(voff: np.ndarray, row_ptr: np.ndarray, width: int = 6) -> np.ndarray:
    """Device bytes a request pins: its graph's row pointers and neighbour
    lists, plus one output row."""
    n = np.diff(voff)
    nnz = row_ptr[voff[1:]] - row_ptr[voff[:-1]]
    return (8 * (n + 1) + 4 * nnz + 8 * width).astype(np.int64)


class Server:
    def __init__(self, batch_handle, footprints: np.ndarray, n_slots: int = 4, max_batch: int = 512,
                 budget_bytes: int = 1 << 30, k: int = 4):
        import torch
        self.b = batch_handle
        self.k = k
        self.fp = np.asarray(footprints, dtype=np.int64)
        self.max_batch = max_batch
        self.budget = int(budget_bytes)
        self.streams = [torch.cuda.Stream() for _ in range(n_slots)]
        self.slots = [binding.pg_batch_slot_create(batch_handle, max_batch, s) for s in self.streams]

    def close(self):
        for s in self.slots:
            binding.pg_batch_slot_free(s)
        self.slots = []

    def run(self, graph_ids: np.ndarray, arrival_s: np.ndarray) -> ServeStats:
        """Serves requests (graph_ids[i] arriving at arrival_s[i] seconds after
        the start, non-decreasing) and returns latencies and results."""
        N = int(graph_ids.shape[0])
        width = 2 if self.k == 3 else 6
        results = np.zeros((N, width), dtype=np.uint64)
        done_at = np.zeros(N, dtype=np.float64)
        pending = deque()
        busy = {}            # slot index -> request indices
        inflight = 0
        max_inflight = 0
        batches = []
        nxt = 0
        completed = 0
        t0 = time.perf_counter()
        while completed < N:
            now = time.perf_counter() - t0
            while nxt < N and arrival_s[nxt] <= now:
                pending.append(nxt)
                nxt += 1
            # completions
            for si in list(busy):
                if binding.pg_batch_slot_query(self.slots[si]):
                    reqs = busy.pop(si)
                    rows = binding.pg_batch_slot_wait(self.slots[si], len(reqs), self.k)
                    t = time.perf_counter() - t0
                    for j, r in enumerate(reqs):
                        results[r] = rows[j]
                        done_at[r] = t
                        inflight -= int(self.fp[graph_ids[r]])
                    completed += len(reqs)
            # admit into idle slots
            for si in range(len(self.slots)):
                if not pending:
                    break
                if si in busy:
                    continue
                take = []
                while pending and len(take) < self.max_batch:
                    r = pending[0]
                    f = int(self.fp[graph_ids[r]])
                    if take and inflight + f > self.budget:
                        break
                    if not take and inflight > 0 and inflight + f > self.budget:
                        break
                    take.append(pending.popleft())
                    inflight += f
                if not take:
                    break
                max_inflight = max(max_inflight, inflight)
                binding.pg_batch_slot_submit(self.slots[si], self.k, graph_ids[np.array(take)])
                busy[si] = take
                batches.append(len(take))
            if not busy and not pending and nxt < N:
                # idle until the next arrival
                wait = arrival_s[nxt] - (time.perf_counter() - t0)
                if wait > 2e-4:
                    time.sleep(wait - 1e-4)
        elapsed = done_at.max() - (arrival_s[0] if N else 0.0)
        lat = 1000.0 * (done_at - arrival_s)
        return ServeStats(N, float(elapsed), N / max(elapsed, 1e-9), float(np.percentile(lat, 50)),
                          float(np.percentile(lat, 99)), float(np.mean(batches)) if batches else 0.0,
                          int(max_inflight), lat, results)


def poisson_arrivals(n: int, rate: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n))
