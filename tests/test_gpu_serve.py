"""Asynchronous slots and the serving loop: every replay of a slot's
captured launch, and every request served in a mix, gives the same counts
as the eager batched call for that graph alone (tolerance 0)."""
import numpy as np
import pytest

from paper_1911_06969_amd import binding, serve, synth
from tests.gpu_common import gpu_or_skip, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return gpu_or_skip()


@pytest.fixture(scope="module")
def loaded(torch):
    b = synth.motif_batch(1500, seed=21)
    h = binding.pg_batch_load(b.voff, b.row_ptr, b.col)
    eager = binding.pg_batch_count_motifs(h, 4, None, n_graphs=b.n_graphs)
    eager3 = binding.pg_batch_count_motifs(h, 3, None, n_graphs=b.n_graphs)
    yield b, h, eager, eager3
    binding.pg_batch_free(h)


def test_slot_replays_match_eager(loaded):
    b, h, eager, eager3 = loaded
    slot = binding.pg_batch_slot_create(h, 64)
    rng = np.random.default_rng(3)
    try:
        for rep in range(6):
            ids = rng.choice(b.n_graphs, int(rng.integers(1, 65)), replace=True)
            k = 4 if rep % 3 else 3
            n = binding.pg_batch_slot_submit(slot, k, ids)
            rows = binding.pg_batch_slot_wait(slot, n, k)
            assert np.array_equal(rows, (eager if k == 4 else eager3)[ids]), rep
            # eager work and a synchronisation between replays
            again = binding.pg_batch_count_motifs(h, 4, ids[:3])
            assert np.array_equal(again, eager[ids[:3]])
    finally:
        binding.pg_batch_slot_free(slot)


def test_two_slots_overlap(torch, loaded):
    b, h, eager, _ = loaded
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    a = binding.pg_batch_slot_create(h, 256, s1)
    c = binding.pg_batch_slot_create(h, 256, s2)
    try:
        ids1 = np.arange(0, 256)
        ids2 = np.arange(1000, 1256)
        binding.pg_batch_slot_submit(a, 4, ids1)
        binding.pg_batch_slot_submit(c, 4, ids2)
        with pytest.raises(binding.PgError):
            binding.pg_batch_slot_submit(a, 4, ids1)   # busy
        r2 = binding.pg_batch_slot_wait(c, 256)
        r1 = binding.pg_batch_slot_wait(a, 256)
        assert np.array_equal(r1, eager[ids1])
        assert np.array_equal(r2, eager[ids2])
        assert binding.pg_batch_slot_query(a)
    finally:
        binding.pg_batch_slot_free(a)
        binding.pg_batch_slot_free(c)


def test_served_results_equal_alone(loaded):
    b, h, eager, _ = loaded
    fp = serve.graph_footprints(b.voff, b.row_ptr)
    srv = serve.Server(h, fp, n_slots=3, max_batch=128, budget_bytes=1 << 30)
    try:
        rng = np.random.default_rng(6)
        ids = rng.integers(0, b.n_graphs, 3000)
        arr = serve.poisson_arrivals(3000, 20000.0, seed=7)
        st = srv.run(ids, arr)
    finally:
        srv.close()
    say("served", st.throughput, st.p50_ms, st.p99_ms, st.mean_batch)
    assert np.array_equal(st.results, eager[ids])
    assert st.p99_ms >= st.p50_ms > 0
    assert st.n_requests == 3000


def test_admission_respects_footprint_budget(loaded):
    b, h, eager, _ = loaded
    fp = serve.graph_footprints(b.voff, b.row_ptr)
    budget = int(fp.max()) * 2
    srv = serve.Server(h, fp, n_slots=4, max_batch=64, budget_bytes=budget)
    try:
        ids = np.arange(0, 400)
        arr = np.zeros(400)   # all at once: admission alone limits the batches
        st = srv.run(ids, arr)
    finally:
        srv.close()
    assert st.max_inflight_bytes <= max(budget, int(fp.max()))
    assert np.array_equal(st.results, eager[ids])


def test_autotuner_grid_keeps_counts(torch, loaded):
    """The autotuner over a 2 x 2 grid (workgroup size x grid size) leaves
    its best parameters on the batch; counts are unchanged for direct calls
    and for a slot that re-captures its launch with them."""
    from paper_1911_06969_amd import tune
    b, h, eager, _ = loaded
    ids = np.arange(0, b.n_graphs, 3)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    rows = []
    slot = binding.pg_batch_slot_create(h, 128)
    try:
        before = binding.pg_batch_slot_submit(slot, 4, ids[:100])
        assert np.array_equal(binding.pg_batch_slot_wait(slot, before), eager[ids[:100]])
        best, table = tune.tune(h, ids, n_cu, repeats=1, log=rows.append, blocks=(128, 512), splits=(2.5e5,),
                                grid_per_cu=(1, 3))
        assert len(table) == 4 and best in table
        say("tuned", best)
        assert np.array_equal(binding.pg_batch_count_motifs(h, 4, ids), eager[ids])
        n = binding.pg_batch_slot_submit(slot, 4, ids[100:228])
        assert np.array_equal(binding.pg_batch_slot_wait(slot, n), eager[ids[100:228]])
        # parameters that differ from the tuned ones, then the slot again
        binding.pg_batch_set_params(h, 64, 1e5, 7)
        n = binding.pg_batch_slot_submit(slot, 4, ids[:50])
        assert np.array_equal(binding.pg_batch_slot_wait(slot, n), eager[ids[:50]])
        assert np.array_equal(binding.pg_batch_count_motifs(h, 4, ids), eager[ids])
    finally:
        binding.pg_batch_slot_free(slot)
        binding.pg_batch_set_params(h, 256, 4e6, 2 * n_cu)
