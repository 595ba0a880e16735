"""Seeded synthetic inputs (R-MAT, Erdos-Renyi, batches, small families).

This module only produces graphs.  It holds none of the mining arithmetic:
it writes the canonical CSR the method assumes (symmetric, loop-free,
duplicate-free, rows ascending; Pangolin section 6.1) and nothing else.
The HIP path and the CPU oracle both read what it returns.

The heavy generators live in ``synth.c`` (counter-based splitmix64 draws,
so the output does not depend on the thread count); the small families
used by the tests are built here in numpy.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None


def build_lib(force: bool = False) -> str:
    """Compile the generator library with gcc (host code only)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_lib()
        lib = ctypes.CDLL(_LIB_PATH)
        i64, i32, dbl, u64, ptr = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_uint64, ctypes.c_void_p
        lib.synth_rmat_pairs.argtypes = [ctypes.c_int, i64, dbl, dbl, dbl, u64, ptr, ptr]
        lib.synth_rmat_pairs.restype = None
        lib.synth_csr_from_pairs.argtypes = [i64, i64, ptr, ptr, ptr, ptr]
        lib.synth_csr_from_pairs.restype = i64
        lib.synth_er_count.argtypes = [i64, dbl, u64]
        lib.synth_er_count.restype = i64
        lib.synth_er_fill.argtypes = [i64, dbl, u64, ptr, ptr]
        lib.synth_er_fill.restype = None
        lib.synth_labels.argtypes = [i64, i32, u64, ptr]
        lib.synth_labels.restype = None
        lib.synth_er_batch_params.argtypes = [i64, i32, i32, dbl, dbl, u64, ptr, ptr, ptr]
        lib.synth_er_batch_params.restype = None
        lib.synth_er_batch_fill.argtypes = [i64, ptr, ptr, u64, ptr, ptr, ptr, ptr]
        lib.synth_er_batch_fill.restype = None
        _lib = lib
    return _lib


def _p(a: np.ndarray) -> int:
    return a.ctypes.data


@dataclass
class CSR:
    """Undirected graph as symmetric CSR (int64 row_ptr, int32 col)."""
    row_ptr: np.ndarray
    col: np.ndarray
    labels: np.ndarray | None = None
    n_labels: int = 0

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def n_edges(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def adj(self, v: int) -> np.ndarray:
        return self.col[self.row_ptr[v]:self.row_ptr[v + 1]]

    def edges(self) -> np.ndarray:
        """Undirected edges (u < v), shape (E, 2), in (u, v) order."""
        src = np.repeat(np.arange(self.n, dtype=np.int64), self.degrees())
        m = src < self.col
        return np.stack([src[m], self.col[m].astype(np.int64)], axis=1)


@dataclass
class Batch:
    """Many small graphs in one CSR: graph g owns vertices voff[g]..voff[g+1]-1
    of ``row_ptr`` (positions into ``col``); ``col`` holds local vertex ids."""
    voff: np.ndarray
    row_ptr: np.ndarray
    col: np.ndarray
    n: np.ndarray
    p: np.ndarray

    @property
    def n_graphs(self) -> int:
        return int(self.voff.shape[0] - 1)

    def graph(self, g: int) -> CSR:
        v0, v1 = int(self.voff[g]), int(self.voff[g + 1])
        rp = self.row_ptr[v0:v1 + 1]
        base = int(rp[0])
        return CSR((rp - base).astype(np.int64), self.col[base:int(rp[-1])].copy())

    def subset(self, idx) -> "Batch":
        parts = [self.graph(int(g)) for g in idx]
        return batch_from_graphs(parts)


# ----------------------------------------------------------------- builders

def from_edges(n: int, edges, labels=None, n_labels: int = 0) -> CSR:
    """Canonical CSR from an undirected edge list (loops/duplicates dropped)."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    e = e[e[:, 0] != e[:, 1]]
    a = np.concatenate([e[:, 0], e[:, 1]])
    b = np.concatenate([e[:, 1], e[:, 0]])
    key = np.unique(a * max(n, 1) + b)
    src = key // max(n, 1)
    dst = (key % max(n, 1)).astype(np.int32)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, src + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.int64)
    lab = None if labels is None else np.asarray(labels, dtype=np.int32)
    return CSR(row_ptr, dst, lab, n_labels)


def rmat(scale: int, edge_factor: int, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 1) -> CSR:
    """Undirected R-MAT graph on 2^scale vertices from edge_factor*2^scale
    sampled pairs, seeded vertex permutation, loops and duplicates removed."""
    lib = _load()
    n = 1 << scale
    m = edge_factor * n
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    lib.synth_rmat_pairs(scale, m, a, b, c, seed, _p(src), _p(dst))
    row_ptr = np.empty(n + 1, dtype=np.int64)
    col = np.empty(2 * m, dtype=np.int32)
    nnz = lib.synth_csr_from_pairs(n, m, _p(src), _p(dst), _p(row_ptr), _p(col))
    del src, dst
    return CSR(row_ptr, col[:nnz].copy())


def erdos_renyi(n: int, p: float, seed: int = 1, n_labels: int = 0) -> CSR:
    """G(n, p) by geometric skipping; optional labels uniform over n_labels."""
    lib = _load()
    m = lib.synth_er_count(n, p, seed)
    row_ptr = np.empty(n + 1, dtype=np.int64)
    col = np.empty(max(2 * m, 1), dtype=np.int32)
    lib.synth_er_fill(n, p, seed, _p(row_ptr), _p(col))
    labels = None
    if n_labels > 0:
        labels = np.empty(n, dtype=np.int32)
        lib.synth_labels(n, n_labels, seed, _p(labels))
    return CSR(row_ptr, col[:2 * m], labels, n_labels)


def random_labels(n: int, n_labels: int, seed: int) -> np.ndarray:
    lib = _load()
    labels = np.empty(n, dtype=np.int32)
    lib.synth_labels(n, n_labels, seed, _p(labels))
    return labels


def er_batch(n_graphs: int, nmin: int = 10, nmax: int = 400, pmin: float = 0.02,
             pmax: float = 0.3, seed: int = 5) -> Batch:
    """Batch of G(n_g, p_g) graphs, n_g ~ U{nmin..nmax}, p_g ~ U[pmin, pmax]."""
    lib = _load()
    G = n_graphs
    ns = np.empty(G, dtype=np.int32)
    ps = np.empty(G, dtype=np.float64)
    ms = np.empty(G, dtype=np.int64)
    lib.synth_er_batch_params(G, nmin, nmax, pmin, pmax, seed, _p(ns), _p(ps), _p(ms))
    voff = np.zeros(G + 1, dtype=np.int64)
    voff[1:] = np.cumsum(ns)
    eoff = np.zeros(G + 1, dtype=np.int64)
    eoff[1:] = np.cumsum(2 * ms)
    row_ptr = np.empty(int(voff[-1]) + 1, dtype=np.int64)
    col = np.empty(max(int(eoff[-1]), 1), dtype=np.int32)
    lib.synth_er_batch_fill(G, _p(ns), _p(ps), seed, _p(voff), _p(eoff), _p(row_ptr), _p(col))
    return Batch(voff, row_ptr, col[:int(eoff[-1])], ns, ps)


def batch_from_graphs(graphs) -> Batch:
    ns = np.array([g.n for g in graphs], dtype=np.int32)
    voff = np.zeros(len(graphs) + 1, dtype=np.int64)
    voff[1:] = np.cumsum(ns)
    rps, cols = [], []
    base = 0
    for g in graphs:
        rps.append(g.row_ptr[:-1] + base)
        cols.append(g.col.astype(np.int32))
        base += g.nnz
    rps.append(np.array([base], dtype=np.int64))
    row_ptr = np.concatenate(rps).astype(np.int64)
    col = np.concatenate(cols) if cols else np.zeros(0, np.int32)
    return Batch(voff, row_ptr, col, ns, np.zeros(len(graphs)))


# ------------------------------------------------------- small graph families

def empty(n: int) -> CSR:
    return from_edges(n, np.zeros((0, 2), np.int64))


def complete(n: int) -> CSR:
    iu = np.triu_indices(n, 1)
    return from_edges(n, np.stack(iu, axis=1))


def star(m: int) -> CSR:
    return from_edges(m + 1, [(0, i) for i in range(1, m + 1)])


def cycle(n: int) -> CSR:
    return from_edges(n, [(i, (i + 1) % n) for i in range(n)])


def path(n: int) -> CSR:
    return from_edges(n, [(i, i + 1) for i in range(n - 1)])


def complete_multipartite(sizes) -> CSR:
    part = np.concatenate([np.full(s, i) for i, s in enumerate(sizes)]) if sizes else np.zeros(0, int)
    n = int(part.shape[0])
    iu = np.triu_indices(n, 1)
    e = np.stack(iu, axis=1)
    e = e[part[e[:, 0]] != part[e[:, 1]]]
    return from_edges(n, e)


def disjoint_union(*gs: CSR) -> CSR:
    edges, off = [], 0
    labs = []
    for g in gs:
        edges.append(g.edges() + off)
        if g.labels is not None:
            labs.append(g.labels)
        off += g.n
    lab = np.concatenate(labs) if len(labs) == len(gs) and labs else None
    return from_edges(off, np.concatenate(edges) if edges else np.zeros((0, 2)), lab,
                      max([g.n_labels for g in gs] + [0]))


def relabel(g: CSR, perm: np.ndarray) -> CSR:
    """Same graph with vertex v renamed perm[v]."""
    e = g.edges()
    lab = None
    if g.labels is not None:
        lab = np.empty_like(g.labels)
        lab[perm] = g.labels
    return from_edges(g.n, perm[e], lab, g.n_labels)


def gnp_small(n: int, p: float, seed: int, n_labels: int = 0) -> CSR:
    """Small G(n, p) drawn with numpy (for exhaustive tests)."""
    rng = np.random.default_rng(seed)
    iu = np.triu_indices(n, 1)
    keep = rng.random(iu[0].shape[0]) < p
    lab = rng.integers(0, n_labels, n).astype(np.int32) if n_labels > 0 else None
    return from_edges(n, np.stack([iu[0][keep], iu[1][keep]], axis=1), lab, n_labels)


def all_graphs(n: int):
    """Every labelled simple graph on n vertices (2^C(n,2) of them)."""
    iu = np.stack(np.triu_indices(n, 1), axis=1)
    for mask in range(1 << iu.shape[0]):
        sel = [(mask >> i) & 1 for i in range(iu.shape[0])]
        yield from_edges(n, iu[np.array(sel, dtype=bool)])


# ------------------------------------------------- the five named workloads

def triangle_rmat(seed: int = 1) -> CSR:
    """R-MAT scale 14 (16,384 vertices), edge factor 8, a=.57 b=.19 c=.19."""
    return rmat(14, 8, seed=seed)


def clique_rmat(seed: int = 2) -> CSR:
    """R-MAT scale 21 (2,097,152 vertices), edge factor 13."""
    return rmat(21, 13, seed=seed)


def motif_rmat(seed: int = 3) -> CSR:
    """R-MAT scale 18 (262,144 vertices), edge factor 8."""
    return rmat(18, 8, seed=seed)


def fsm_er(seed: int = 4, n: int = 500_000, avg_degree: float = 8.0, n_labels: int = 16) -> CSR:
    """Labelled G(n, p) with p = avg_degree/(n-1), labels uniform over 16."""
    return erdos_renyi(n, avg_degree / (n - 1), seed=seed, n_labels=n_labels)


def motif_batch(n_graphs: int = 100_000, seed: int = 5) -> Batch:
    """Small G(n_g, p_g): n_g ~ U{10..400}, p_g ~ U[0.02, 0.3]."""
    return er_batch(n_graphs, 10, 400, 0.02, 0.3, seed)
