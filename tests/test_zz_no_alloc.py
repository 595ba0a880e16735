"""The allocation-free batch entry point (pg_batch_count_motifs_noalloc)
against pg_batch_count_motifs: same rows, exact integers, on two calls in a
row (the second smaller, so stale rows of the first would show), for k = 4
and k = 3, plus the size limit."""
import numpy as np
import pytest

from paper_1911_06969_amd import binding, synth
from tests.gpu_common import gpu_or_skip, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return gpu_or_skip()


def _batch():
    rng = np.random.default_rng(21)
    graphs = [synth.gnp_small(int(rng.integers(10, 200)), float(rng.uniform(0.02, 0.3)), 100 + s)
              for s in range(300)]
    graphs += [synth.complete(40), synth.star(300), synth.empty(3), synth.erdos_renyi(512, 0.3, seed=3)]
    return synth.batch_from_graphs(graphs)


def test_noalloc_matches_batch_two_calls(torch):
    b = _batch()
    h = binding.pg_batch_load(b.voff, b.row_ptr, b.col)
    try:
        rng = np.random.default_rng(5)
        big = rng.permutation(b.n_graphs)[:250]
        small = np.array([b.n_graphs - 1, 3, 3, 0, b.n_graphs - 2], dtype=np.int64)
        for k in (4, 3):
            for ids in (big, small):
                say(f"noalloc k={k} n_ids={ids.shape[0]}")
                want = binding.pg_batch_count_motifs(h, k, ids)
                got = binding.pg_batch_count_motifs_noalloc(h, k, ids)
                assert got.shape == want.shape
                assert np.array_equal(got, want), (k, ids.shape[0])
        # the whole batch (ids == NULL) and an empty id list
        want = binding.pg_batch_count_motifs(h, 4, None, n_graphs=b.n_graphs)
        got = binding.pg_batch_count_motifs_noalloc(h, 4, None, n_graphs=b.n_graphs)
        assert np.array_equal(got, want)
        assert binding.pg_batch_count_motifs_noalloc(h, 4, np.zeros(0, np.int64)).shape == (0, 6)
    finally:
        binding.pg_batch_free(h)


def test_noalloc_rejects_too_many_ids(torch):
    b = synth.batch_from_graphs([synth.complete(5)])
    h = binding.pg_batch_load(b.voff, b.row_ptr, b.col)
    try:
        ids = np.zeros(binding.PG_BATCH_STATIC_MAX_IDS + 1, dtype=np.int64)
        with pytest.raises(binding.PgError) as e:
            binding.pg_batch_count_motifs_noalloc(h, 4, ids)
        assert e.value.code == binding.PG_EINVAL
        with pytest.raises(binding.PgError) as e:
            binding.pg_batch_count_motifs_noalloc(h, 5, np.zeros(1, np.int64))
        assert e.value.code == binding.PG_EUNSUPPORTED
        # a call at the limit still works
        ids = np.zeros(binding.PG_BATCH_STATIC_MAX_IDS, dtype=np.int64)
        got = binding.pg_batch_count_motifs_noalloc(h, 4, ids)
        assert np.all(got[:, 5] == 5) and np.all(got[:, :5] == 0)
    finally:
        binding.pg_batch_free(h)
