"""GPU parity of motif counting (pg_count_motifs) against the CPU oracle
(brute force on tiny graphs, ESU and the closed form beyond).  Exact
integer counts: the bar is equality."""
from math import comb

import numpy as np
import pytest

import oracle
from oracle import brute, closed_form
from paper_1911_06969_amd import binding, synth
from tests.gpu_common import golden, gpu_or_skip, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return gpu_or_skip()


def gpu_motifs(g, k, budget=None):
    with binding.Graph.from_csr(g) as G:
        if budget:
            G.set_memory_budget(budget)
        return [int(x) for x in G.motifs(k)]


def test_every_graph_on_five_vertices(torch):
    for g in synth.all_graphs(5):
        for k in (3, 4):
            assert gpu_motifs(g, k) == [int(x) for x in brute.motif_counts(g, k)]


@pytest.mark.parametrize("seed", range(16))
def test_brute_force_small(torch, seed):
    rng = np.random.default_rng(300 + seed)
    g = synth.gnp_small(int(rng.integers(5, 13)), float(rng.uniform(0.1, 0.9)), seed)
    for k in (3, 4):
        assert gpu_motifs(g, k) == [int(x) for x in brute.motif_counts(g, k)]


def test_families(torch):
    assert gpu_motifs(synth.star(40), 4) == [0, comb(40, 3), 0, 0, 0, 0]
    assert gpu_motifs(synth.star(40), 3) == [comb(40, 2), 0]
    assert gpu_motifs(synth.cycle(50), 4) == [50, 0, 0, 0, 0, 0]
    assert gpu_motifs(synth.cycle(4), 4) == [0, 0, 1, 0, 0, 0]
    assert gpu_motifs(synth.path(30), 4) == [27, 0, 0, 0, 0, 0]
    assert gpu_motifs(synth.complete(12), 4) == [0, 0, 0, 0, 0, comb(12, 4)]
    assert gpu_motifs(synth.complete(12), 3) == [0, comb(12, 3)]
    a, b = 7, 9
    assert gpu_motifs(synth.complete_multipartite([a, b]), 4) == [
        0, a * comb(b, 3) + b * comb(a, 3), comb(a, 2) * comb(b, 2), 0, 0, 0]
    assert gpu_motifs(synth.empty(10), 4) == [0] * 6
    assert gpu_motifs(synth.empty(0), 3) == [0] * 2


def test_hub_lists_beyond_lds_stage(torch):
    """A star with 2000 leaves plus a dense core: adjacency lists longer than
    the LDS stage and common-neighbour lists longer than its LDS copy."""
    core = synth.complete(40)
    hub = synth.star(2000)
    g = synth.disjoint_union(core, hub, synth.erdos_renyi(1500, 0.05, seed=3))
    for k in (3, 4):
        want = closed_form.motif3(g) if k == 3 else closed_form.motif4(g)
        assert gpu_motifs(g, k) == [int(x) for x in want]


def test_dense_shared_neighbourhoods(torch):
    # degrees ~680 (> LDS stage), common-neighbour lists ~540 (> their LDS copy)
    g = synth.erdos_renyi(850, 0.8, seed=4)
    assert gpu_motifs(g, 4) == [int(x) for x in closed_form.motif4(g)]


@pytest.mark.parametrize("scale,ef,seed", [(9, 8, 1), (11, 8, 2), (12, 16, 3)])
def test_rmat_against_oracle(torch, scale, ef, seed):
    g = synth.rmat(scale, ef, seed=seed)
    for k in (3, 4):
        want = closed_form.motif3(g) if k == 3 else closed_form.motif4(g)
        say("rmat", scale, ef, k, list(want))
        assert gpu_motifs(g, k) == [int(x) for x in want]


def test_esu_on_rmat(torch):
    g = synth.rmat(9, 6, seed=8)
    for k in (3, 4):
        assert gpu_motifs(g, k) == [int(x) for x in oracle.motif_esu(g, k)]


def test_edge_blocking_same_counts(torch):
    g = synth.rmat(11, 8, seed=6)
    want = [int(x) for x in closed_form.motif4(g)]
    assert gpu_motifs(g, 4, budget=1 << 20) == want


def test_relabel_invariance(torch):
    g = synth.rmat(10, 8, seed=7)
    h = synth.relabel(g, np.random.default_rng(2).permutation(g.n))
    assert gpu_motifs(g, 4) == gpu_motifs(h, 4)


def test_reduce_example_triangles_and_wedge(torch):
    """Three embeddings reduce to {triangle: 2, wedge: 1} (section 3.1)."""
    g = synth.disjoint_union(synth.complete(3), synth.complete(3), synth.path(3))
    assert gpu_motifs(g, 3) == [1, 2]


def test_automorphism_example_counted_once(torch):
    """(3,5,4) and (2,5,4) both extend to {2,3,4,5} (section 3.2): the 4-set
    is counted once.  Graph: 5 adjacent to 2, 3 and 4; 4 adjacent to 3."""
    g = synth.from_edges(6, [(5, 2), (5, 3), (5, 4), (4, 3)])
    # {2,3,4,5}: edges 52 53 54 43 -> paw
    assert gpu_motifs(g, 4) == [0, 0, 0, 1, 0, 0]


def test_triangle_rmat_config(torch):
    g = synth.triangle_rmat()
    want = golden("full_configs.json")["triangle_rmat_s14"]
    assert gpu_motifs(g, 3) == want["motif3"]
    assert gpu_motifs(g, 4) == want["motif4"]


@pytest.mark.slow
def test_motif_rmat_config(torch):
    """R-MAT scale 18, edge factor 8: the motif workload at full size."""
    g = synth.motif_rmat()
    want = golden("full_configs.json")["motif_rmat_s18"]
    with binding.Graph.from_csr(g) as G:
        say("scale-18 k=3")
        assert [int(x) for x in G.motifs(3)] == want["motif3"]
        say("scale-18 k=4")
        assert [int(x) for x in G.motifs(4)] == want["motif4"]


def test_binary_search_connectivity_example(torch):
    """The connectivity check of section 5 (binary search figure): embedding
    {2, 5, 8} (here the path 2-5-8) and candidate 9, whose neighbour list
    holds 2 and 5 but not 8.  The 4-set {2, 5, 8, 9} is then a triangle
    2-5-9 with the pendant 8 (a paw), the only connected 4-set."""
    g = synth.from_edges(10, [(2, 5), (5, 8), (2, 9), (5, 9)])
    assert gpu_motifs(g, 4) == [0, 0, 0, 1, 0, 0]
    assert gpu_motifs(g, 4) == [int(x) for x in brute.motif_counts(g, 4)]
    assert gpu_motifs(g, 3) == [int(x) for x in brute.motif_counts(g, 3)]


@pytest.mark.parametrize("n_total", [60_000, 70_000, 200_000, 300_000, 600_000])
def test_map_kernel_sizes(torch, n_total):
    """4-motifs on graphs whose vertex count selects each size of the
    workgroup's two-bit vertex map (up to 2^16, 2^17, 2^18, 2^19 vertices)
    and one beyond it (per-wave kernel only): a hub of degree 3000, a dense
    random block and isolated vertices, against the closed form."""
    parts = [synth.star(3000), synth.erdos_renyi(700, 0.4, seed=11), synth.rmat(11, 8, seed=5)]
    used = sum(p.n for p in parts)
    g = synth.disjoint_union(*parts, synth.empty(n_total - used))
    assert g.n == n_total
    want = [int(x) for x in closed_form.motif4(g)]
    say("map sizes", n_total, want)
    assert gpu_motifs(g, 4) == want


def test_map_kernel_shared_hub_and_threshold(torch):
    """Entries just below and above the many-children threshold (255, 256
    and 257 leaves beyond a shared pair), a complete bipartite K_{2,300}
    (two hubs sharing every neighbour) and a budget small enough to cut the
    level-2 list into many chunks."""
    parts = [synth.complete_multipartite([2, 300])]
    for leaves in (255, 256, 257, 513):
        parts.append(synth.star(leaves))
    g = synth.disjoint_union(*parts, synth.erdos_renyi(700, 0.5, seed=9))
    want = [int(x) for x in closed_form.motif4(g)]
    a, b = 2, 300
    kab = [0, a * comb(b, 3) + b * comb(a, 3), comb(a, 2) * comb(b, 2), 0, 0, 0]
    assert [int(x) for x in closed_form.motif4(parts[0])] == kab
    assert gpu_motifs(g, 4) == want
    assert gpu_motifs(g, 4, budget=1 << 20) == want
