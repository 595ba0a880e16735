"""ctypes binding of libpangolin_hip.so (argument marshalling only).

Every function keeps the C name of the entry point it wraps
(include/pangolin_hip.h) and does no mining work itself: host arrays are
passed as numpy buffers, device arrays as torch tensors on the GPU (their
data pointers, with PG_DEVICE_PTRS).  A missing or unloadable library
raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpangolin_hip.so")

PG_OK, PG_EINVAL, PG_ENOMEM, PG_EUNSUPPORTED, PG_EDEVICE, PG_EOVERFLOW = 0, -1, -2, -3, -4, -5
PG_DEVICE_PTRS = 1
PG_CANONICALIZE = 2
PG_KMAX = 8
PG_BATCH_MAX_VERTICES = 512

EXPORTS = (
    "pg_graph_load_csr", "pg_graph_free", "pg_graph_set_stream", "pg_graph_info",
    "pg_set_memory_budget", "pg_graph_set_option", "pg_count_cliques", "pg_list_cliques", "pg_count_motifs",
    "pg_fsm",
    "pg_fsm_num_patterns", "pg_fsm_pattern_key", "pg_batch_load", "pg_batch_free",
    "pg_batch_count_motifs", "pg_batch_count_motifs_noalloc", "pg_batch_slot_create", "pg_batch_slot_submit", "pg_batch_slot_query",
    "pg_batch_slot_wait", "pg_batch_slot_free", "pg_batch_work_estimate",
    "pg_batch_set_params", "pg_last_error", "pg_set_allocator", "pg_profile_enable",
    "pg_profile_reset", "pg_profile_query", "pg_profile_list", "pg_version",
)

_lib = None


class PgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pangolin_hip error {code}: {msg}")
        self.code = code


def load_library(path: str | None = None):
    """Loads the HIP library (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise ImportError(f"{path} not built; run __graft_entry__.build() or "
                          "python paper_1911_06969_amd/build.py")
    lib = ctypes.CDLL(path)
    i64, u64, i32, cint, ptr, sz = (ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int,
                                    ctypes.c_void_p, ctypes.c_size_t)
    P = ctypes.POINTER
    lib.pg_graph_load_csr.argtypes = [i64, i64, ptr, ptr, ptr, i32, ctypes.c_uint, ptr, P(ptr)]
    lib.pg_graph_free.argtypes = [ptr]
    lib.pg_graph_set_stream.argtypes = [ptr, ptr]
    lib.pg_graph_info.argtypes = [ptr, P(i64), P(i64), P(i64)]
    lib.pg_set_memory_budget.argtypes = [ptr, u64]
    lib.pg_graph_set_option.argtypes = [ptr, cint, i64]
    lib.pg_count_cliques.argtypes = [ptr, cint, P(u64)]
    lib.pg_list_cliques.argtypes = [ptr, cint, ptr, u64, P(u64)]
    lib.pg_count_motifs.argtypes = [ptr, cint, ptr]
    lib.pg_fsm.argtypes = [ptr, cint, u64, ptr, sz, P(sz)]
    lib.pg_fsm_num_patterns.argtypes = [cint, cint]
    lib.pg_fsm_num_patterns.restype = u64
    lib.pg_fsm_pattern_key.argtypes = [u64, cint, cint, P(cint), ptr]
    lib.pg_batch_load.argtypes = [i64, ptr, ptr, ptr, ctypes.c_uint, ptr, P(ptr)]
    lib.pg_batch_free.argtypes = [ptr]
    lib.pg_batch_count_motifs.argtypes = [ptr, cint, ptr, i64, ptr]
    lib.pg_batch_count_motifs_noalloc.argtypes = [ptr, cint, ptr, i64, ptr]
    lib.pg_batch_slot_create.argtypes = [ptr, i64, ptr, P(ptr)]
    lib.pg_batch_slot_submit.argtypes = [ptr, cint, ptr, i64]
    lib.pg_batch_slot_query.argtypes = [ptr]
    lib.pg_batch_slot_wait.argtypes = [ptr, ptr]
    lib.pg_batch_slot_free.argtypes = [ptr]
    lib.pg_batch_work_estimate.argtypes = [ptr, ptr]
    lib.pg_batch_set_params.argtypes = [ptr, cint, ctypes.c_double, cint]
    lib.pg_last_error.restype = ctypes.c_char_p
    lib.pg_set_allocator.argtypes = [ptr, ptr, ptr]
    lib.pg_profile_enable.argtypes = [cint]
    lib.pg_profile_query.argtypes = [ctypes.c_char_p, P(ctypes.c_double), P(u64), P(ctypes.c_double)]
    lib.pg_profile_list.argtypes = [ctypes.c_char_p, sz]
    lib.pg_version.restype = ctypes.c_char_p
    for name in EXPORTS:
        f = getattr(lib, name)
        if name not in ("pg_fsm_num_patterns", "pg_last_error", "pg_version"):
            f.restype = cint
    _lib = lib
    if os.environ.get("PG_ALLOCATOR", "torch") == "torch":
        use_torch_allocator()
    return lib


_ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_torch_hooks = None


def use_torch_allocator() -> bool:
    """Routes the library's device allocations through torch's caching
    allocator (pg_set_allocator), so that graphs, levels and batches share
    torch's memory pool.  Done by load_library unless PG_ALLOCATOR=hip; a
    no-op without a GPU.  Returns whether the hooks are installed."""
    global _torch_hooks
    try:
        import torch
    except ImportError:
        return False
    if not torch.cuda.is_available():
        return False

    def alloc(nbytes, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes))
        except RuntimeError:
            return None

    def free(p, ctx):
        torch.cuda.caching_allocator_delete(int(p))

    hooks = (_ALLOC(alloc), _FREE(free))
    if _lib.pg_set_allocator(hooks[0], hooks[1], None) != PG_OK:
        return False
    _torch_hooks = hooks   # the callbacks must outlive every allocation
    return True


def _check(rc: int):
    if rc != PG_OK:
        msg = load_library().pg_last_error().decode(errors="replace")
        raise PgError(rc, msg)


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


def _dev_ptr(t, dtype_name: str):
    if str(t.dtype) != dtype_name:
        raise TypeError(f"expected {dtype_name}, got {t.dtype}")
    if not t.is_cuda or not t.is_contiguous():
        raise TypeError("device arrays must be contiguous GPU tensors")
    return ctypes.c_void_p(t.data_ptr())


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, ctypes.c_void_p(a.ctypes.data)


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


# ---------------------------------------------------------------- graphs

def pg_graph_load_csr(row_ptr, col_idx, labels=None, n_labels: int = 0, stream=None, canonicalize: bool = False):
    """Loads a CSR graph (numpy host arrays or torch GPU tensors).  Returns
    the opaque handle.  canonicalize: PG_CANONICALIZE (the library sorts,
    symmetrises and drops loops and duplicates)."""
    lib = load_library()
    dev = _is_torch(row_ptr)
    keep = []
    if dev:
        n = row_ptr.shape[0] - 1
        nnz = col_idx.shape[0]
        prp, pcol = _dev_ptr(row_ptr, "torch.int64"), _dev_ptr(col_idx, "torch.int32")
        plab = _dev_ptr(labels, "torch.int32") if labels is not None else None
        flags = PG_DEVICE_PTRS
    else:
        rp, prp = _host(row_ptr, np.int64)
        col, pcol = _host(col_idx, np.int32)
        keep += [rp, col]
        n, nnz = rp.shape[0] - 1, col.shape[0]
        plab = None
        if labels is not None:
            lab, plab = _host(labels, np.int32)
            keep.append(lab)
        flags = 0
    if canonicalize:
        flags |= PG_CANONICALIZE
    out = ctypes.c_void_p()
    _check(lib.pg_graph_load_csr(n, nnz, prp, pcol, plab, n_labels if labels is not None else 0, flags,
                                 _stream_ptr(stream), ctypes.byref(out)))
    return out


def pg_graph_free(g) -> None:
    _check(load_library().pg_graph_free(g))


def pg_graph_set_stream(g, stream) -> None:
    _check(load_library().pg_graph_set_stream(g, _stream_ptr(stream)))


def pg_graph_info(g):
    n, nnz, dmax = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(load_library().pg_graph_info(g, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(dmax)))
    return n.value, nnz.value, dmax.value


def pg_set_memory_budget(g, nbytes: int) -> None:
    _check(load_library().pg_set_memory_budget(g, int(nbytes)))


PG_OPT_CLIQUE_MASKS = 1
PG_OPT_FSM_BIT_KEYS = 2


def pg_graph_set_option(g, option: int, value: int) -> None:
    _check(load_library().pg_graph_set_option(g, int(option), int(value)))


def pg_count_cliques(g, k: int) -> int:
    c = ctypes.c_uint64()
    _check(load_library().pg_count_cliques(g, int(k), ctypes.byref(c)))
    return int(c.value)


def pg_list_cliques(g, k: int, capacity: int):
    """(rows, total): the first min(total, capacity) k-cliques as an int32
    array of shape (rows, k), and the number of k-cliques."""
    out = np.zeros((max(int(capacity), 0), int(k)), dtype=np.int32)
    t = ctypes.c_uint64()
    p = ctypes.c_void_p(out.ctypes.data) if out.size else None
    _check(load_library().pg_list_cliques(g, int(k), p, int(capacity), ctypes.byref(t)))
    return out[:min(int(t.value), out.shape[0])], int(t.value)


MOTIF_CLASSES = {3: 2, 4: 6, 5: 21}


def pg_count_motifs(g, k: int) -> np.ndarray:
    out = np.zeros(21, dtype=np.uint64)
    _check(load_library().pg_count_motifs(g, int(k), ctypes.c_void_p(out.ctypes.data)))
    return out[: MOTIF_CLASSES.get(int(k), 0)]


def pg_fsm_num_patterns(max_edges: int, n_labels: int) -> int:
    return int(load_library().pg_fsm_num_patterns(int(max_edges), int(n_labels)))


def pg_fsm(g, max_edges: int, min_support: int, n_labels: int):
    """Returns (supports, n_frequent); supports is indexed by the dense
    pattern index, 0 for infrequent patterns."""
    npat = pg_fsm_num_patterns(max_edges, n_labels)
    sup = np.zeros(max(npat, 1), dtype=np.uint64)
    nf = ctypes.c_size_t()
    _check(load_library().pg_fsm(g, int(max_edges), int(min_support), ctypes.c_void_p(sup.ctypes.data),
                                 sup.shape[0], ctypes.byref(nf)))
    return sup[:npat], int(nf.value)


def pg_fsm_pattern_key(index: int, max_edges: int, n_labels: int):
    shape = ctypes.c_int()
    lab = np.zeros(5, dtype=np.int32)
    _check(load_library().pg_fsm_pattern_key(int(index), int(max_edges), int(n_labels), ctypes.byref(shape),
                                             ctypes.c_void_p(lab.ctypes.data)))
    return int(shape.value), [int(x) for x in lab if x >= 0]


# --------------------------------------------------------------- batches

def pg_batch_load(voff, row_ptr, col, stream=None):
    lib = load_library()
    vo, pvo = _host(voff, np.int64)
    if _is_torch(row_ptr):
        prp, pcol = _dev_ptr(row_ptr, "torch.int64"), _dev_ptr(col, "torch.int32")
        flags = PG_DEVICE_PTRS
        keep = [vo]
    else:
        rp, prp = _host(row_ptr, np.int64)
        cl, pcol = _host(col, np.int32)
        keep = [vo, rp, cl]
        flags = 0
    out = ctypes.c_void_p()
    _check(lib.pg_batch_load(vo.shape[0] - 1, pvo, prp, pcol, flags, _stream_ptr(stream), ctypes.byref(out)))
    del keep
    return out


def pg_batch_free(b) -> None:
    _check(load_library().pg_batch_free(b))


def pg_batch_count_motifs(b, k: int, ids=None, n_graphs: int | None = None) -> np.ndarray:
    lib = load_library()
    width = 2 if k == 3 else 6
    if ids is None:
        if n_graphs is None:
            raise ValueError("n_graphs is needed when ids is None")
        out = np.zeros((n_graphs, width), dtype=np.uint64)
        _check(lib.pg_batch_count_motifs(b, int(k), None, 0, ctypes.c_void_p(out.ctypes.data)))
        return out
    idv, pid = _host(ids, np.int64)
    out = np.zeros((idv.shape[0], width), dtype=np.uint64)
    _check(lib.pg_batch_count_motifs(b, int(k), pid, idv.shape[0], ctypes.c_void_p(out.ctypes.data)))
    return out


PG_BATCH_STATIC_MAX_IDS = 16384


def pg_batch_count_motifs_noalloc(b, k: int, ids=None, n_graphs: int | None = None) -> np.ndarray:
    """pg_batch_count_motifs through the allocation-free entry point (at most
    PG_BATCH_STATIC_MAX_IDS graphs per call)."""
    lib = load_library()
    width = 2 if k == 3 else 6
    if ids is None:
        if n_graphs is None:
            raise ValueError("n_graphs is needed when ids is None")
        out = np.zeros((n_graphs, width), dtype=np.uint64)
        _check(lib.pg_batch_count_motifs_noalloc(b, int(k), None, 0, ctypes.c_void_p(out.ctypes.data)))
        return out
    idv, pid = _host(ids, np.int64)
    out = np.zeros((idv.shape[0], width), dtype=np.uint64)
    _check(lib.pg_batch_count_motifs_noalloc(b, int(k), pid, idv.shape[0], ctypes.c_void_p(out.ctypes.data)))
    return out


def pg_batch_slot_create(b, max_ids: int, stream=None):
    out = ctypes.c_void_p()
    _check(load_library().pg_batch_slot_create(b, int(max_ids), _stream_ptr(stream), ctypes.byref(out)))
    return out


def pg_batch_slot_submit(slot, k: int, ids) -> int:
    """Enqueues the counts of ids (host int64 array); returns the number of
    ids submitted.  The id array is copied before the call returns."""
    idv, pid = _host(ids, np.int64)
    _check(load_library().pg_batch_slot_submit(slot, int(k), pid, idv.shape[0]))
    return int(idv.shape[0])


def pg_batch_slot_query(slot) -> bool:
    rc = load_library().pg_batch_slot_query(slot)
    if rc < 0:
        _check(rc)
    return rc == 1


def pg_batch_slot_wait(slot, n_ids: int, k: int = 4) -> np.ndarray:
    out = np.zeros((max(n_ids, 1), 2 if k == 3 else 6), dtype=np.uint64)
    _check(load_library().pg_batch_slot_wait(slot, ctypes.c_void_p(out.ctypes.data)))
    return out[:n_ids]


def pg_batch_slot_free(slot) -> None:
    _check(load_library().pg_batch_slot_free(slot))


def pg_batch_work_estimate(b, n_graphs: int) -> np.ndarray:
    out = np.zeros(n_graphs, dtype=np.float64)
    _check(load_library().pg_batch_work_estimate(b, ctypes.c_void_p(out.ctypes.data)))
    return out


def pg_batch_set_params(b, block_threads: int = 0, split_work: float = 0.0, grid_blocks: int = 0) -> None:
    _check(load_library().pg_batch_set_params(b, int(block_threads), float(split_work), int(grid_blocks)))


# --------------------------------------------------------------- runtime

def pg_last_error() -> str:
    return load_library().pg_last_error().decode(errors="replace")


def pg_version() -> str:
    return load_library().pg_version().decode()


def pg_profile_enable(on: bool = True) -> None:
    _check(load_library().pg_profile_enable(1 if on else 0))


def pg_profile_reset() -> None:
    _check(load_library().pg_profile_reset())


def pg_profile_query(kernel: str):
    """(total_ms, launches, units) for a kernel, or None if it never ran."""
    ms, n, u = ctypes.c_double(), ctypes.c_uint64(), ctypes.c_double()
    rc = load_library().pg_profile_query(kernel.encode(), ctypes.byref(ms), ctypes.byref(n), ctypes.byref(u))
    if rc != PG_OK:
        return None
    return ms.value, int(n.value), u.value


def pg_profile_list() -> list:
    buf = ctypes.create_string_buffer(1 << 16)
    _check(load_library().pg_profile_list(buf, len(buf)))
    return [s for s in buf.value.decode().split("\n") if s]


# ------------------------------------------------------------- helpers

class Graph:
    """Owns a pg_graph handle."""

    def __init__(self, row_ptr, col_idx, labels=None, n_labels: int = 0, stream=None, canonicalize: bool = False):
        self.n_labels = n_labels if labels is not None else 0
        self.h = pg_graph_load_csr(row_ptr, col_idx, labels, n_labels, stream, canonicalize)

    @classmethod
    def from_csr(cls, g, stream=None, canonicalize: bool = False):
        return cls(g.row_ptr, g.col, g.labels, g.n_labels, stream, canonicalize)

    def info(self):
        """(vertices, directed entries, maximum degree)."""
        return pg_graph_info(self.h)

    def cliques(self, k: int) -> int:
        return pg_count_cliques(self.h, k)

    def list_cliques(self, k: int, capacity: int):
        return pg_list_cliques(self.h, k, capacity)

    def motifs(self, k: int) -> np.ndarray:
        return pg_count_motifs(self.h, k)

    def fsm(self, max_edges: int, min_support: int):
        return pg_fsm(self.h, max_edges, min_support, self.n_labels)

    def set_memory_budget(self, nbytes: int) -> None:
        pg_set_memory_budget(self.h, nbytes)

    def set_option(self, option: int, value: int) -> None:
        pg_graph_set_option(self.h, option, value)

    def close(self) -> None:
        if self.h is not None:
            pg_graph_free(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
