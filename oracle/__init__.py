"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct computations of what the mining path
computes, written from the definitions in Pangolin (VLDB 2020).  Only the
tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this package.  It shares no code with the HIP library.

Layers:
  * ``oracle.cpp`` (built to ``liboracle.so`` with g++/OpenMP): clique
    enumeration in the degree order, ESU motif enumeration, closed-form
    pieces, edge-subset enumeration with domain (MNI) support for patterns
    of up to four edges (pattern index by enumerated tables).
  * ``brute.py``: brute force over vertex subsets and over injective maps,
    for graphs of a dozen vertices.
  * ``closed_form.py``: exact 4-motif counts from non-induced counts.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build_lib(force: bool = False) -> str:
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_lib()
        lib = ctypes.CDLL(_LIB_PATH)
        i64, u64, ptr, cint = ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int
        lib.or_max_threads.restype = cint
        lib.or_clique_count.argtypes = [i64, ptr, ptr, cint, cint]
        lib.or_clique_count.restype = u64
        lib.or_clique_count_roots.argtypes = [i64, ptr, ptr, cint, ptr, i64, ptr, cint]
        lib.or_clique_count_roots.restype = u64
        lib.or_motif_esu.argtypes = [i64, ptr, ptr, cint, ptr, cint]
        lib.or_motif_esu.restype = None
        lib.or_motif_esu_roots.argtypes = [i64, ptr, ptr, cint, ptr, i64, ptr, cint]
        lib.or_motif_esu_roots.restype = None
        lib.or_motif_parts.argtypes = [i64, ptr, ptr, ptr, cint]
        lib.or_motif_parts.restype = None
        lib.or_fsm_num_patterns.argtypes = [cint, cint]
        lib.or_fsm_num_patterns.restype = u64
        lib.or_fsm_pattern_index.argtypes = [cint, ptr, cint]
        lib.or_fsm_pattern_index.restype = u64
        lib.or_fsm_supports.argtypes = [i64, ptr, ptr, ptr, cint, cint, ptr, ptr, cint]
        lib.or_fsm_supports.restype = cint
        _lib = lib
    return _lib


def _c(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data


def max_threads() -> int:
    return int(_load().or_max_threads())


def clique_count(g, k: int, nthreads: int = 0) -> int:
    """Number of k-cliques (k-subsets pairwise adjacent)."""
    rp, prp = _c(g.row_ptr, np.int64)
    col, pcol = _c(g.col, np.int32)
    return int(_load().or_clique_count(g.n, prp, pcol, k, nthreads))


def clique_list(g, k: int) -> list:
    """Every k-clique as its ascending tuple of vertex ids, in lexicographic
    order (section 2.2 k-cliques; section 3.3 listing).  Plain ordered
    extension: a clique (v1 < ... < vj) grows by each common neighbour of
    all its vertices that is larger than vj.  For graphs with up to about
    10^6 cliques."""
    nbr = [set(int(u) for u in g.adj(v)) for v in range(g.n)]
    out = []

    def grow(clique, cand):
        if len(clique) == k:
            out.append(tuple(clique))
            return
        for u in sorted(cand):
            grow(clique + [u], {w for w in cand if w > u and w in nbr[u]})

    if k >= 1:
        grow([], set(range(g.n)))
    return out


def clique_count_roots(g, k: int, roots, nthreads: int = 0):
    """k-cliques whose first vertex in the degree order is each given root."""
    rp, prp = _c(g.row_ptr, np.int64)
    col, pcol = _c(g.col, np.int32)
    r, pr = _c(roots, np.int64)
    out = np.zeros(r.shape[0], dtype=np.uint64)
    _load().or_clique_count_roots(g.n, prp, pcol, k, pr, r.shape[0], out.ctypes.data, nthreads)
    return out


MOTIF3_NAMES = ("wedge", "triangle")
MOTIF4_NAMES = ("path", "star", "cycle", "paw", "diamond", "clique")


MOTIF_CLASSES = {3: 2, 4: 6, 5: 21}


def motif_esu(g, k: int, nthreads: int = 0) -> np.ndarray:
    """Induced k-motif counts (k = 3: wedge, triangle; k = 4: path, star,
    cycle, paw, diamond, 4-clique; k = 5: the 21 connected graphs in the
    order of ``brute.motif5_classes``) by ESU enumeration."""
    assert k in MOTIF_CLASSES
    rp, prp = _c(g.row_ptr, np.int64)
    col, pcol = _c(g.col, np.int32)
    out = np.zeros(21, dtype=np.uint64)
    _load().or_motif_esu(g.n, prp, pcol, k, out.ctypes.data, nthreads)
    return out[: MOTIF_CLASSES[k]]


def motif_esu_roots(g, k: int, roots, nthreads: int = 0) -> np.ndarray:
    """ESU restricted to connected subsets whose smallest vertex is a root."""
    assert k in MOTIF_CLASSES
    rp, prp = _c(g.row_ptr, np.int64)
    col, pcol = _c(g.col, np.int32)
    r, pr = _c(roots, np.int64)
    out = np.zeros(21, dtype=np.uint64)
    _load().or_motif_esu_roots(g.n, prp, pcol, k, pr, r.shape[0], out.ctypes.data, nthreads)
    return out[: MOTIF_CLASSES[k]]


def motif_parts(g, nthreads: int = 0) -> dict:
    rp, prp = _c(g.row_ptr, np.int64)
    col, pcol = _c(g.col, np.int32)
    out = np.zeros(7, dtype=np.uint64)
    _load().or_motif_parts(g.n, prp, pcol, out.ctypes.data, nthreads)
    keys = ("wedges_noninduced", "triangles", "stars_noninduced", "p4_raw",
            "c4_twice", "paws_noninduced", "diamonds_noninduced")
    return {k: int(v) for k, v in zip(keys, out)}


FSM_SHAPES = ("edge", "wedge", "triangle", "path4", "star3", "path5", "star4", "fork", "cycle4", "paw")


def fsm_num_patterns(max_edges: int, n_labels: int) -> int:
    """Size of the dense index of labelled patterns with 1..max_edges edges
    (max_edges <= 4), counted by enumerating the label tuples of each shape."""
    return int(_load().or_fsm_num_patterns(max_edges, n_labels))


def fsm_pattern_index(shape: int, labels, n_labels: int) -> int:
    """Dense index of the pattern of `shape` whose positions carry `labels`
    (any of the tuples naming it)."""
    lab, pl = _c(list(labels) + [0] * (5 - len(labels)), np.int32)
    return int(_load().or_fsm_pattern_index(shape, pl, n_labels))


def fsm_supports_all(g, max_edges: int, nthreads: int = 0):
    """Unfiltered MNI support of every labelled pattern with 1..max_edges
    edges (max_edges <= 4) at its dense index, and the number of embeddings
    per size."""
    assert g.labels is not None and g.n_labels > 0
    rp, prp = _c(g.row_ptr, np.int64)
    col, pcol = _c(g.col, np.int32)
    lab, plab = _c(g.labels, np.int32)
    npat = fsm_num_patterns(max_edges, g.n_labels)
    sup = np.zeros(npat, dtype=np.uint64)
    cnt = np.zeros(4, dtype=np.uint64)
    rc = _load().or_fsm_supports(g.n, prp, pcol, plab, g.n_labels, max_edges,
                                 sup.ctypes.data, cnt.ctypes.data, nthreads)
    if rc != 0:
        raise ValueError("unsupported max_edges or label count")
    return sup, cnt[:max_edges]


def fsm(g, max_edges: int, min_support: int, nthreads: int = 0) -> np.ndarray:
    """Supports of the frequent patterns (support >= min_support), 0 for
    the others (Pangolin's FSM prunes when support < MIN_SUPPORT)."""
    sup, _ = fsm_supports_all(g, max_edges, nthreads)
    out = sup.copy()
    out[sup < np.uint64(max(min_support, 0))] = 0
    return out
