"""Host-side checks of the C-ABI library: it loads, exports every symbol
the header declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

from paper_1911_06969_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pangolin_hip.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(binding.LIB_PATH):
        from paper_1911_06969_amd import build
        build.build(verbose=False)
    return binding.load_library()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pg_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("pg_graph_load_csr", "pg_count_cliques", "pg_count_motifs", "pg_fsm", "pg_batch_count_motifs"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_names_match_header():
    assert set(binding.EXPORTS) == set(declared_functions())


def test_null_arguments_rejected(lib):
    c = ctypes.c_uint64()
    assert lib.pg_count_cliques(None, 3, ctypes.byref(c)) == binding.PG_EINVAL
    assert lib.pg_count_motifs(None, 4, None) == binding.PG_EINVAL
    assert lib.pg_list_cliques(None, 3, None, 0, ctypes.byref(c)) == binding.PG_EINVAL
    # a non-zero capacity needs rows to write into
    assert lib.pg_list_cliques(ctypes.c_void_p(8), 3, None, 5, ctypes.byref(c)) == binding.PG_EINVAL
    assert "NULL" in binding.pg_last_error()
    assert lib.pg_graph_free(None) == binding.PG_OK


def test_unsupported_sizes_rejected(lib):
    c = ctypes.c_uint64()
    # size checks come before any device access
    assert lib.pg_count_cliques(ctypes.c_void_p(8), 0, ctypes.byref(c)) == binding.PG_EUNSUPPORTED
    assert lib.pg_count_cliques(ctypes.c_void_p(8), 9, ctypes.byref(c)) == binding.PG_EUNSUPPORTED
    assert lib.pg_list_cliques(ctypes.c_void_p(8), 9, None, 0, ctypes.byref(c)) == binding.PG_EUNSUPPORTED


def test_version(lib):
    assert "gfx950" in binding.pg_version()


def test_no_device_fails_loudly(lib):
    """Without a GPU the library refuses to run rather than falling back."""
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("GPU present")
    except ImportError:
        pass
    with pytest.raises(binding.PgError) as e:
        binding.pg_graph_load_csr([0, 1, 2], [1, 0])
    assert e.value.code == binding.PG_EDEVICE


def test_fsm_pattern_count_matches_format(lib):
    assert binding.pg_fsm_num_patterns(3, 16) == 49080
    assert binding.pg_fsm_num_patterns(1, 16) == 136
    assert binding.pg_fsm_num_patterns(2, 16) == 136 + 16 * 136
    assert binding.pg_fsm_num_patterns(5, 16) == 0


def test_fsm_pattern_keys_decode_the_dense_index(lib):
    """The library's decoder and the oracle's enumerated table agree on the
    documented pattern numbering (shape blocks, lexicographic labels)."""
    from oracle import brute
    L = 3
    for i, (shape, lab) in enumerate(brute.pattern_table(3, L)):
        got_shape, got_lab = binding.pg_fsm_pattern_key(i, 3, L)
        assert (got_shape, tuple(got_lab)) == (shape, tuple(lab))


def test_fsm_four_edge_index(lib):
    """Patterns of up to four edges: the index size equals the oracle's
    enumeration for several label counts, and the decoder walks the
    enumerated table of the oracle's brute-force module."""
    import oracle
    from oracle import brute
    for L in (1, 2, 3, 5, 16, 32):
        assert binding.pg_fsm_num_patterns(4, L) == oracle.fsm_num_patterns(4, L), L
    assert binding.pg_fsm_num_patterns(4, 33) == 0
    L = 3
    table = brute.pattern_table(4, L)
    assert len(table) == binding.pg_fsm_num_patterns(4, L)
    for i, (shape, lab) in enumerate(table):
        got_shape, got_lab = binding.pg_fsm_pattern_key(i, 4, L)
        assert (got_shape, tuple(got_lab)) == (shape, tuple(lab)), i
