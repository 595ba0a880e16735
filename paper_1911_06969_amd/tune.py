"""Autotuner for the batched motif kernel's tile and work-split parameters.

Times pg_batch_count_motifs over a sample of the batch for every
combination of workgroup size, split threshold (estimated work above which
a graph becomes several queue items) and persistent grid size, and returns
the fastest.  The result can be stored as JSON and applied with
pg_batch_set_params.
"""
from __future__ import annotations

import itertools
import json
import time

import numpy as np

from . import binding

BLOCKS = (128, 256, 512)
SPLITS = (2.5e5, 1e6, 4e6, 1.6e7)
GRID_PER_CU = (1, 2, 4)


def tune(batch_handle, ids: np.ndarray, n_cu: int, k: int = 4, repeats: int = 2, log=None,
         blocks=BLOCKS, splits=SPLITS, grid_per_cu=GRID_PER_CU):
    """Grid search; leaves the fastest parameters set on the batch and
    returns (best, table)."""
    best = None
    table = []
    for bt, sp, gpc in itertools.product(blocks, splits, grid_per_cu):
        binding.pg_batch_set_params(batch_handle, bt, sp, gpc * n_cu)
        binding.pg_batch_count_motifs(batch_handle, k, ids)   # warm-up
        t = time.perf_counter()
        for _ in range(repeats):
            binding.pg_batch_count_motifs(batch_handle, k, ids)
        dt = (time.perf_counter() - t) / repeats
        row = {"block_threads": bt, "split_work": sp, "grid_blocks": gpc * n_cu, "seconds": dt}
        table.append(row)
        if log:
            log(row)
        if best is None or dt < best["seconds"]:
            best = row
    binding.pg_batch_set_params(batch_handle, best["block_threads"], best["split_work"], best["grid_blocks"])
    return best, table


def save(path: str, best: dict, table: list, note: str = "") -> None:
    with open(path, "w") as f:
        json.dump({"best": best, "table": table, "note": note}, f, indent=1)


def load(path: str):
    with open(path) as f:
        return json.load(f)["best"]
