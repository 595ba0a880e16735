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
            binding.pg_fsm(G.h, 4, 1, 1)
        assert e.value.code == binding.PG_EUNSUPPORTED


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
