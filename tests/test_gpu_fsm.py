"""GPU parity of frequent subgraph mining (pg_fsm) against the CPU oracle:
supports from injective maps by definition on tiny graphs, edge-subset
enumeration with domain sets beyond.  Exact integers: the bar is equality."""
import hashlib

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_1911_06969_amd import binding, synth
from tests.gpu_common import golden, gpu_or_skip, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return gpu_or_skip()


def gpu_fsm(g, max_edges, sigma, budget=None):
    with binding.Graph.from_csr(g) as G:
        if budget:
            G.set_memory_budget(budget)
        sup, nf = G.fsm(max_edges, sigma)
    assert nf == int((sup > 0).sum())
    return sup


@pytest.mark.parametrize("seed", range(12))
def test_against_injective_maps(torch, seed):
    rng = np.random.default_rng(400 + seed)
    L = int(rng.integers(1, 4))
    g = synth.gnp_small(int(rng.integers(5, 10)), float(rng.uniform(0.2, 0.7)), seed, n_labels=L)
    for sigma in (0, 1, 2, 3):
        for K in (1, 2, 3):
            want = brute.fsm(g, K, sigma)
            assert np.array_equal(gpu_fsm(g, K, sigma), want), (seed, sigma, K)


def test_single_label_edge_support(torch):
    g = synth.rmat(10, 4, seed=41)
    g = synth.CSR(g.row_ptr, g.col, np.zeros(g.n, np.int32), 1)
    sup = gpu_fsm(g, 1, 1)
    assert int(sup[0]) == int((g.degrees() > 0).sum())


@pytest.mark.parametrize("n,p,L,sigma", [(3000, 8 / 2999, 4, 50), (2000, 0.004, 3, 1), (4000, 0.003, 6, 20),
                                         (800, 0.02, 2, 400)])
def test_er_against_oracle(torch, n, p, L, sigma):
    g = synth.erdos_renyi(n, p, seed=42, n_labels=L)
    for K in (1, 2, 3):
        want = oracle.fsm(g, K, sigma)
        got = gpu_fsm(g, K, sigma)
        say("er", n, L, sigma, K, int((want > 0).sum()))
        assert np.array_equal(got, want)


def test_largest_label_alphabet(torch):
    """64 labels, the most a graph may carry: 11.5 million pattern slots
    for up to 3 edges, label ranks up to ~60 per class."""
    g = synth.erdos_renyi(3000, 0.004, seed=47, n_labels=64)
    for K in (1, 2, 3):
        for sigma in (1, 3):
            assert np.array_equal(gpu_fsm(g, K, sigma), oracle.fsm(g, K, sigma)), (K, sigma)


def test_power_law_labelled(torch):
    g = synth.rmat(11, 8, seed=43)
    g = synth.CSR(g.row_ptr, g.col, synth.random_labels(g.n, 5, 44), 5)
    for sigma in (10, 100):
        assert np.array_equal(gpu_fsm(g, 3, sigma), oracle.fsm(g, 3, sigma))


def test_bitmap_groups_under_small_budget(torch):
    g = synth.erdos_renyi(20000, 8 / 19999, seed=45, n_labels=8)
    want = oracle.fsm(g, 3, 5)
    assert np.array_equal(gpu_fsm(g, 3, 5, budget=8 << 20), want)


@pytest.mark.parametrize("n,L,sigma", [(30000, 6, 20), (5000, 3, 2)])
def test_bit_keys_and_atomic_bits_agree(torch, n, L, sigma):
    """Domain bits of three-edge patterns through sorted keys (the default)
    and through atomic ORs give the oracle's supports."""
    g = synth.erdos_renyi(n, 8 / (n - 1), seed=46, n_labels=L)
    want = oracle.fsm(g, 3, sigma)
    for keys in (1, 0):
        with binding.Graph.from_csr(g) as G:
            G.set_option(binding.PG_OPT_FSM_BIT_KEYS, keys)
            sup, nf = binding.pg_fsm(G.h, 3, sigma, g.n_labels)
        say("fsm bit keys", keys, n, L, sigma, nf)
        assert np.array_equal(sup, want)


def test_thresholds_and_antimonotone(torch):
    g = synth.erdos_renyi(3000, 0.003, seed=46, n_labels=3)
    allsup = gpu_fsm(g, 3, 0)
    none = gpu_fsm(g, 3, 10 ** 12)
    assert not none.any()
    mid = gpu_fsm(g, 3, 30)
    assert np.array_equal(mid, np.where(allsup >= 30, allsup, 0))


def test_rejects_unlabelled_and_bad_sizes(torch):
    g = synth.rmat(8, 4, seed=47)
    with binding.Graph.from_csr(g) as G:
        with pytest.raises(binding.PgError) as e:
            binding.pg_fsm(G.h, 3, 1, 4)
        assert e.value.code == binding.PG_EINVAL
    g.labels = np.zeros(g.n, np.int32)
    g.n_labels = 1
    with binding.Graph.from_csr(g) as G:
        with pytest.raises(binding.PgError) as e:
            binding.pg_fsm(G.h, 5, 1, 1)
        assert e.value.code == binding.PG_EUNSUPPORTED
    g.labels = (np.arange(g.n) % 33).astype(np.int32)
    g.n_labels = 33
    with binding.Graph.from_csr(g) as G:
        # four edges need at most 32 labels
        with pytest.raises(binding.PgError) as e:
            binding.pg_fsm(G.h, 4, 1, 33)
        assert e.value.code in (binding.PG_EUNSUPPORTED, binding.PG_EINVAL)


@pytest.mark.slow
def test_fsm_er_config(torch):
    """Labelled G(n, p), 500k vertices, average degree 8, 16 labels, sigma 1000,
    patterns of up to 3 edges."""
    g = synth.fsm_er()
    want = golden("full_configs.json")["fsm_er_500k"]["sigma1000"]
    sup = gpu_fsm(g, 3, 1000)
    say("fsm full", int((sup > 0).sum()))
    assert int((sup > 0).sum()) == want["n_frequent"]
    assert int(sup.sum()) == want["sum"]
    assert [int(sup[i]) for i in want["sample_index"]] == want["sample_support"]
    assert hashlib.sha256(sup.astype(np.uint64).tobytes()).hexdigest() == want["sha256"]


@pytest.mark.parametrize("seed", range(10))
def test_four_edges_against_injective_maps(torch, seed):
    """Patterns of four edges (5-path, 4-star, fork, 4-cycle, paw) on tiny
    graphs: supports by definition from injective maps."""
    rng = np.random.default_rng(900 + seed)
    L = int(rng.integers(1, 4))
    g = synth.gnp_small(int(rng.integers(5, 10)), float(rng.uniform(0.25, 0.7)), 50 + seed, n_labels=L)
    for sigma in (0, 1, 2, 3):
        want = brute.fsm(g, 4, sigma)
        say(f"fsm4 brute seed={seed} n={g.n} L={L} sigma={sigma}")
        assert np.array_equal(gpu_fsm(g, 4, sigma), want), (seed, sigma)


def test_four_edge_shapes_one_by_one(torch):
    """Each four-edge shape alone with distinct and with equal labels: its
    pattern's support is the smallest orbit's domain."""
    shapes = {
        "path5": [(0, 1), (1, 2), (2, 3), (3, 4)],
        "star4": [(0, 1), (0, 2), (0, 3), (0, 4)],
        "fork": [(0, 1), (0, 2), (0, 3), (3, 4)],
        "cycle4": [(0, 1), (1, 2), (2, 3), (3, 0)],
        "paw": [(0, 1), (0, 2), (0, 3), (2, 3)],
    }
    for name, edges in shapes.items():
        n = 1 + max(max(e) for e in edges)
        for labels in (np.zeros(n, np.int32), np.arange(n, dtype=np.int32) % 3):
            L = int(labels.max()) + 1
            g = synth.from_edges(n, edges)
            g = synth.CSR(g.row_ptr, g.col, labels, L)
            want = brute.fsm(g, 4, 1)
            assert np.array_equal(gpu_fsm(g, 4, 1), want), (name, labels)


@pytest.mark.parametrize("n,p,L,sigma", [(1500, 6 / 1499, 3, 40), (2500, 0.002, 4, 5), (500, 0.016, 2, 60)])
def test_four_edges_er_against_oracle(torch, n, p, L, sigma):
    g = synth.erdos_renyi(n, p, seed=61, n_labels=L)
    want = oracle.fsm(g, 4, sigma)
    say("fsm4 er", n, L, sigma, int((want > 0).sum()))
    assert np.array_equal(gpu_fsm(g, 4, sigma), want)


def test_four_edges_power_law_and_small_budget(torch):
    """A skewed graph (hub lists, many embeddings per pattern) and a budget
    that forces the level-4 domain bitmaps into several groups."""
    g = synth.rmat(8, 2, seed=62)
    g = synth.CSR(g.row_ptr, g.col, synth.random_labels(g.n, 3, 63), 3)
    want = oracle.fsm(g, 4, 20)
    assert np.array_equal(gpu_fsm(g, 4, 20), want)
    assert np.array_equal(gpu_fsm(g, 4, 20, budget=1 << 20), want)
