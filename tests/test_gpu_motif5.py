"""GPU parity of 5-vertex motif counting (pg_count_motifs with k = 5)
against the CPU oracle: brute force over vertex subsets on tiny graphs, ESU
beyond, closed forms on graph families.  Exact integer counts: the bar is
equality."""
from math import comb

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_1911_06969_amd import binding, synth
from tests.gpu_common import gpu_or_skip, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return gpu_or_skip()


def gpu_motifs(g, budget=None):
    with binding.Graph.from_csr(g) as G:
        if budget:
            G.set_memory_budget(budget)
        return [int(x) for x in G.motifs(5)]


def _class_of(edges) -> int:
    c = brute.motif_counts(synth.from_edges(5, edges), 5)
    return int(np.argmax(c))


def test_every_graph_on_five_vertices(torch):
    for g in synth.all_graphs(5):
        assert gpu_motifs(g) == [int(x) for x in brute.motif_counts(g, 5)]


@pytest.mark.parametrize("seed", range(12))
def test_brute_force_small(torch, seed):
    rng = np.random.default_rng(700 + seed)
    g = synth.gnp_small(int(rng.integers(6, 14)), float(rng.uniform(0.15, 0.9)), seed)
    say(f"motif5 brute n={g.n} seed={seed}")
    assert gpu_motifs(g) == [int(x) for x in brute.motif_counts(g, 5)]


def test_families(torch):
    star = _class_of([(0, 1), (0, 2), (0, 3), (0, 4)])
    path = _class_of([(0, 1), (1, 2), (2, 3), (3, 4)])
    cyc = _class_of([(0, 1), (1, 2), (2, 3), (3, 4), (4, 0)])
    k23 = _class_of([(a, b) for a in (0, 1) for b in (2, 3, 4)])

    def one(slot, value):
        v = [0] * 21
        v[slot] = value
        return v

    assert gpu_motifs(synth.complete(12)) == one(20, comb(12, 5))
    assert gpu_motifs(synth.star(30)) == one(star, comb(30, 4))
    assert gpu_motifs(synth.cycle(40)) == one(path, 40)
    assert gpu_motifs(synth.cycle(5)) == one(cyc, 1)
    assert gpu_motifs(synth.path(20)) == one(path, 16)
    a, b = 6, 7
    want = [0] * 21
    want[star] = a * comb(b, 4) + b * comb(a, 4)
    want[k23] = comb(a, 2) * comb(b, 3) + comb(a, 3) * comb(b, 2)
    assert gpu_motifs(synth.complete_multipartite([a, b])) == want
    assert gpu_motifs(synth.empty(10)) == [0] * 21
    assert gpu_motifs(synth.empty(0)) == [0] * 21


def test_rmat_against_esu(torch):
    """Vertices of degree up to 90: level-1 entries with more than 64
    children (several work items, a ragged last one)."""
    g = synth.rmat(8, 4, seed=1)
    say("motif5 rmat(8, 4) seed 1")
    want = [int(x) for x in oracle.motif_esu(g, 5)]
    assert gpu_motifs(g) == want
    # edge blocking: level 2 in many chunks under a small memory budget
    assert gpu_motifs(g, budget=1 << 20) == want


def test_er_against_esu(torch):
    g = synth.erdos_renyi(400, 0.025, seed=11)
    say("motif5 er(400, 0.025) seed 11")
    assert gpu_motifs(g) == [int(x) for x in oracle.motif_esu(g, 5)]


def test_relabel_invariance(torch):
    g = synth.rmat(9, 4, seed=7)
    h = synth.relabel(g, np.random.default_rng(3).permutation(g.n))
    assert gpu_motifs(g) == gpu_motifs(h)


def test_bench_workload_against_esu(torch):
    """The measured workload at full size: G(n,p), n = 100,000, average
    degree 8, seed 12 (about 4.3e8 embeddings), against the oracle's ESU."""
    n = 100_000
    g = synth.erdos_renyi(n, 8.0 / (n - 1), seed=12)
    say("motif5 bench workload: er(100000, d=8) seed 12")
    got = gpu_motifs(g)
    assert got == [int(x) for x in oracle.motif_esu(g, 5)]
    assert sum(got) > 4 * 10**8


def test_hub_lists_beyond_the_stage(torch):
    """Hubs of degree above 256, whose lists are not staged in LDS: a star of
    300 leaves with the hub first (v0) and last (v1) in vertex order, and a
    complete bipartite K_{2,300} (two hubs sharing every neighbour), against
    closed forms."""
    star = _class_of([(0, 1), (0, 2), (0, 3), (0, 4)])
    k23 = _class_of([(a, b) for a in (0, 1) for b in (2, 3, 4)])
    s = synth.star(300)
    one = [0] * 21
    one[star] = comb(300, 4)
    assert gpu_motifs(s) == one
    perm = np.arange(s.n)
    perm[0], perm[-1] = perm[-1], perm[0]          # hub named 300
    assert gpu_motifs(synth.relabel(s, perm)) == one
    a, b = 2, 300
    want = [0] * 21
    want[star] = a * comb(b, 4) + b * comb(a, 4)
    want[k23] = comb(a, 2) * comb(b, 3) + comb(a, 3) * comb(b, 2)
    assert gpu_motifs(synth.complete_multipartite([a, b])) == want


@pytest.mark.slow
def test_sparse_graph_with_hub_against_esu(torch):
    """A sparse G(n, p) with one added hub of degree 270 (lists of v0, v1
    and mixed staged/unstaged pairs), class by class against the oracle's
    ESU."""
    base = synth.erdos_renyi(3000, 3.0 / 2999, seed=21)
    rng = np.random.default_rng(22)
    hub = base.n
    nbrs = np.sort(rng.choice(base.n, 270, replace=False))
    edges = [(int(u), int(v)) for u in range(base.n) for v in base.col[base.row_ptr[u]:base.row_ptr[u + 1]] if u < v]
    edges += [(int(v), hub) for v in nbrs]
    g = synth.from_edges(base.n + 1, edges)
    say("motif5 sparse + hub 270")
    want = [int(x) for x in oracle.motif_esu(g, 5)]
    assert gpu_motifs(g) == want
