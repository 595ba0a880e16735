"""GPU parity of k-clique counting (pg_count_cliques) against the CPU oracle.
Exact integer counts: the bar is equality."""
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


def gpu_cliques(g, ks, budget=None):
    """Counts through both 4-clique paths (sibling masks and the general
    level kernels); they must agree before the result is compared."""
    out = []
    for masks in (1, 0):
        with binding.Graph.from_csr(g) as G:
            if budget:
                G.set_memory_budget(budget)
            G.set_option(binding.PG_OPT_CLIQUE_MASKS, masks)
            out.append([G.cliques(k) for k in ks])
    assert out[0] == out[1], out
    return out[0]


def test_complete_graphs(torch):
    for n in (1, 2, 3, 4, 7, 12, 20):
        g = synth.complete(n)
        say("K", n)
        assert gpu_cliques(g, range(1, 9)) == [comb(n, k) for k in range(1, 9)]


def test_mask_row_width_limit(torch):
    """K_769: the lowest-ranked vertex has DAG out-degree 768, the most the
    sibling masks take (12-word rows, the deepest search of the count pass);
    in K_770 that vertex (out-degree 769) is a heavy root, counted through
    wide rows in device memory, and the rest by the masks.  K_130 takes
    3-word rows through the deeper mask levels.  Every count against
    C(n, k)."""
    for n, ks in ((769, (3, 4)), (770, (3, 4)), (130, (3, 4, 5, 6))):
        say("K", n)
        assert gpu_cliques(synth.complete(n), ks) == [comb(n, k) for k in ks]


def test_heavy_and_light_roots(torch):
    """K_780 beside an R-MAT graph: the 12 lowest-ranked vertices of K_780
    have DAG out-degrees 779 .. 768, so 11 roots are heavy (wide rows) and
    all others light (sibling masks); the counts add up."""
    k_part = synth.complete(780)
    r_part = synth.rmat(11, 16, seed=8)
    g = synth.disjoint_union(k_part, r_part)
    ks = (3, 4)
    want = [comb(780, k) + oracle.clique_count(r_part, k) for k in ks]
    assert gpu_cliques(g, ks) == want


def test_wide_rows_for_heavy_roots(torch):
    """Heavy roots of out-degree up to 2099 (rows of up to 33 words, both
    register halves of a lane) beside an R-MAT graph: triangles and
    4-cliques through the wide rows equal C(n, k) plus the oracle's count;
    on a smaller pair the general kernels alone agree."""
    parts = [synth.complete(1300), synth.complete(2100), synth.rmat(12, 16, seed=9)]
    g = synth.disjoint_union(*parts)
    ks = (3, 4)
    want = [comb(1300, k) + comb(2100, k) + oracle.clique_count(parts[2], k) for k in ks]
    say("wide rows", want)
    assert gpu_cliques(g, ks) == want
    small = synth.disjoint_union(synth.complete(900), synth.rmat(10, 8, seed=9))
    with binding.Graph.from_csr(small) as G:
        masks = [G.cliques(k) for k in ks]
        G.set_option(binding.PG_OPT_CLIQUE_MASKS, 0)
        assert [G.cliques(k) for k in ks] == masks


def test_wide_rows_under_a_small_budget(torch):
    """When the heavy roots' rows do not fit half the budget, they take the
    general kernels: same counts."""
    g = synth.disjoint_union(synth.complete(900), synth.rmat(10, 8, seed=10))
    want = [comb(900, k) + oracle.clique_count(synth.rmat(10, 8, seed=10), k) for k in (3, 4)]
    with binding.Graph.from_csr(g) as G:
        G.set_memory_budget(1 << 20)
        assert [G.cliques(k) for k in (3, 4)] == want


@pytest.mark.slow
def test_rmat_weak_scaling_sweep(torch):
    """The weak-scaling graphs (R-MAT, edge factor 10, seed 7, 2^20 .. 2^25
    vertices): triangles at every scale and 4-cliques up to scale 23,
    against the oracle's counts."""
    gold = golden("full_configs.json")
    for sc in range(20, 26):
        want = gold[f"rmat_sweep_s{sc}"]
        g = synth.rmat(sc, 10, seed=7)
        assert (g.n, g.n_edges) == (want["n"], want["edges"])
        with binding.Graph.from_csr(g) as G:
            for k in (3, 4):
                if f"k{k}" in want:
                    got = G.cliques(k)
                    say(f"sweep scale {sc} k={k}: {got}")
                    assert got == want[f"k{k}"], (sc, k)
        del g


def test_empty_and_edge_cases(torch):
    assert gpu_cliques(synth.empty(5), [1, 2, 3, 4]) == [5, 0, 0, 0]
    assert gpu_cliques(synth.empty(0), [1, 3]) == [0, 0]
    assert gpu_cliques(synth.path(2), [2, 3]) == [1, 0]
    g = synth.disjoint_union(synth.complete(6), synth.empty(50), synth.star(30))
    assert gpu_cliques(g, [3, 4, 5, 6]) == [comb(6, 3), comb(6, 4), comb(6, 5), 1]


@pytest.mark.parametrize("seed", range(12))
def test_brute_force_small(torch, seed):
    rng = np.random.default_rng(seed)
    g = synth.gnp_small(int(rng.integers(4, 13)), float(rng.uniform(0.2, 0.9)), seed)
    want = [brute.clique_count(g, k) for k in (3, 4, 5)]
    assert gpu_cliques(g, (3, 4, 5)) == want


@pytest.mark.parametrize("sizes", [[2, 3, 4], [5, 5, 5, 5], [1, 7, 2, 9, 3]])
def test_complete_multipartite(torch, sizes):
    import itertools
    g = synth.complete_multipartite(sizes)
    want = [sum(int(np.prod(c)) for c in itertools.combinations(sizes, k)) for k in (3, 4, 5)]
    assert gpu_cliques(g, (3, 4, 5)) == want


@pytest.mark.parametrize("scale,ef,seed", [(9, 8, 1), (11, 16, 2), (12, 8, 3)])
def test_rmat_against_oracle(torch, scale, ef, seed):
    g = synth.rmat(scale, ef, seed=seed)
    ks = (3, 4, 5, 6)
    want = [oracle.clique_count(g, k) for k in ks]
    say("rmat", scale, ef, want)
    assert gpu_cliques(g, ks) == want


def test_dense_random_spans_many_tiles(torch):
    # sibling lists longer than one wave and than the LDS stage
    g = synth.erdos_renyi(3000, 0.2, seed=9)
    ks = (3, 4)
    want = [oracle.clique_count(g, k) for k in ks]
    assert gpu_cliques(g, ks) == want


def test_edge_blocking_same_counts(torch):
    """A tiny memory budget forces the embedding levels into many chunks."""
    g = synth.rmat(12, 16, seed=4)
    ks = (4, 5)
    want = [oracle.clique_count(g, k) for k in ks]
    assert gpu_cliques(g, ks, budget=1 << 20) == want


def test_deeper_levels_under_a_small_budget(torch):
    """k = 6 and 7 store the levels up to k - 3 in chunks under a 4 MiB
    budget; the last mask level then takes each chunk's entries as parents
    and finds their children in the parents' sets."""
    g = synth.rmat(12, 16, seed=4)
    ks = (5, 6, 7)
    want = [oracle.clique_count(g, k) for k in ks]
    say("rmat 12 16, k = 5..7 at 4 MiB", want)
    assert gpu_cliques(g, ks, budget=4 << 20) == want


def test_last_mask_level_on_wide_rows(torch):
    """5-cliques of K_705 and K_769 through the sibling masks: rows of 11
    and 12 words (the odd width reads the word after a row's last), every
    pair of words non-empty; against C(n, 5)."""
    for n in (705, 769):
        say("K", n, "k = 5")
        with binding.Graph.from_csr(synth.complete(n)) as G:
            G.set_option(binding.PG_OPT_CLIQUE_MASKS, 1)
            assert G.cliques(5) == comb(n, 5)


def test_relabel_invariance(torch):
    g = synth.rmat(11, 8, seed=5)
    h = synth.relabel(g, np.random.default_rng(1).permutation(g.n))
    assert gpu_cliques(g, (3, 4, 5)) == gpu_cliques(h, (3, 4, 5))


def test_device_pointer_input(torch):
    g = synth.rmat(10, 8, seed=6)
    rp = torch.from_numpy(g.row_ptr).cuda()
    col = torch.from_numpy(g.col).cuda()
    stream = torch.cuda.current_stream()
    with binding.Graph(rp, col, stream=stream) as G:
        assert G.cliques(4) == oracle.clique_count(g, 4)


def test_invalid_csr_rejected(torch):
    bad = [
        ([0, 1, 1], [1]),                 # not symmetric
        ([0, 1, 2], [0, 1]),              # self-loops
        ([0, 2, 3, 4], [2, 1, 0, 0]),     # unsorted row
        ([0, 1, 2], [5, 0]),              # out of range
        ([0, 2, 1], [1, 0]),              # row_ptr decreasing
    ]
    for rp, col in bad:
        with pytest.raises(binding.PgError) as e:
            binding.Graph(np.array(rp), np.array(col))
        assert e.value.code == binding.PG_EINVAL


def test_triangle_rmat_config(torch):
    """R-MAT scale 14, edge factor 8 (triangle counting workload)."""
    g = synth.triangle_rmat()
    want = golden("full_configs.json")["triangle_rmat_s14"]
    with binding.Graph.from_csr(g) as G:
        assert G.cliques(3) == want["k3"]
        assert G.cliques(4) == want["k4"]


@pytest.mark.slow
def test_clique_rmat_config_k4(torch):
    """R-MAT scale 21, edge factor 13: the k-clique workload at full size."""
    g = synth.clique_rmat()
    want = golden("full_configs.json")["clique_rmat_s21"]
    with binding.Graph.from_csr(g) as G:
        say("scale-21 k=3")
        assert G.cliques(3) == want["k3"]
        say("scale-21 k=4, sibling masks")
        assert G.cliques(4) == want["k4"]
        G.set_option(binding.PG_OPT_CLIQUE_MASKS, 0)
        say("scale-21 k=4, general kernels")
        assert G.cliques(4) == want["k4"]


@pytest.mark.slow
def test_clique_rmat_config_edge_blocking(torch):
    """The scale-21 4-clique count with the level memory bounded to 1.5 GiB
    (the 3.6 GB triangle level goes in about a dozen chunks)."""
    g = synth.clique_rmat()
    want = golden("full_configs.json")["clique_rmat_s21"]
    with binding.Graph.from_csr(g) as G:
        G.set_memory_budget(3 << 29)
        assert G.cliques(4) == want["k4"]


@pytest.mark.slow
def test_clique_rmat_config_k5(torch):
    """R-MAT scale 21: the 5-clique count at full size on the mask levels,
    with the default level budget and with 8 GiB (the 4-clique level, 143 GB,
    then goes in about twenty chunks)."""
    g = synth.clique_rmat()
    want = golden("full_configs.json")["clique_rmat_s21_k5"]
    with binding.Graph.from_csr(g) as G:
        say("scale-21 k=5, sibling masks")
        assert G.cliques(5) == want["k5"]
        G.set_memory_budget(8 << 30)
        say("scale-21 k=5, sibling masks, 8 GiB")
        assert G.cliques(5) == want["k5"]


# ------------------------------------------------------------ clique listing

def _row_sets(rows):
    return sorted(tuple(sorted(r)) for r in rows.tolist())


def test_list_complete_graphs(torch):
    import itertools
    for n in (1, 2, 5, 9):
        g = synth.complete(n)
        with binding.Graph.from_csr(g) as G:
            for k in range(1, min(n, 6) + 1):
                rows, total = G.list_cliques(k, comb(n, k))
                assert total == comb(n, k)
                assert rows.shape == (comb(n, k), k)
                assert _row_sets(rows) == list(itertools.combinations(range(n), k))


@pytest.mark.parametrize("scale,ef,seed", [(8, 8, 1), (10, 8, 2)])
def test_list_rmat_against_oracle(torch, scale, ef, seed):
    g = synth.rmat(scale, ef, seed=seed)
    with binding.Graph.from_csr(g) as G:
        for k in (2, 3, 4, 5):
            want = oracle.clique_list(g, k)
            say("rmat", scale, "k", k, len(want))
            rows, total = G.list_cliques(k, len(want) + 5)
            again, total2 = G.list_cliques(k, len(want) + 5)
            assert total == total2 == len(want)
            assert np.array_equal(rows, again)   # the same rows in the same order
            assert _row_sets(rows) == want


def test_list_capacity_and_edge_blocking(torch):
    """A short buffer gets the first rows of the full listing; capacity 0
    only counts; a tiny memory budget (many chunks) lists the same rows in
    the same order."""
    g = synth.rmat(10, 16, seed=3)
    with binding.Graph.from_csr(g) as G:
        none, total = G.list_cliques(4, 0)
        full, t1 = G.list_cliques(4, total)
        part, t2 = G.list_cliques(4, 1000)
        G.set_memory_budget(1 << 20)
        blocked, t3 = G.list_cliques(4, total)
    assert total == t1 == t2 == t3 == oracle.clique_count(g, 4)
    assert none.shape == (0, 4)
    assert np.array_equal(part, full[:1000])
    assert np.array_equal(blocked, full)
    assert _row_sets(full) == oracle.clique_list(g, 4)


def test_every_graph_on_five_vertices(torch):
    """All 1,024 labelled graphs on five vertices: k-clique counts through
    both paths against brute force, and the listed cliques as sets."""
    for g in synth.all_graphs(5):
        want = [brute.clique_count(g, k) for k in (3, 4, 5)]
        assert gpu_cliques(g, (3, 4, 5)) == want
        with binding.Graph.from_csr(g) as G:
            for k in (2, 3, 4):
                rows, total = G.list_cliques(k, 16)
                assert total == len(rows)
                assert _row_sets(rows) == brute.clique_list(g, k)



def _messy(g, rng):
    """The same edges as a CSR with one direction of some edges missing,
    duplicated entries, self-loops and unsorted rows."""
    rows = []
    for v in range(g.n):
        nb = [int(u) for u in g.col[g.row_ptr[v]:g.row_ptr[v + 1]] if u > v or rng.random() < 0.5]
        nb += [int(u) for u in rng.choice(nb, size=min(len(nb), 2))] if nb else []
        if rng.random() < 0.2:
            nb.append(v)
        rng.shuffle(nb)
        rows.append(nb)
    rp = np.zeros(g.n + 1, np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.array([u for r in rows for u in r], np.int32)
    return rp, col


def test_canonicalize_rebuilds_the_csr(torch):
    """PG_CANONICALIZE: an unsorted, partly one-directional CSR with
    duplicates and loops loads as the canonical CSR of its symmetric closure
    (entry count as the definition gives it), and mines like it."""
    rng = np.random.default_rng(31)
    g = synth.rmat(10, 8, seed=31)
    rp, col = _messy(g, rng)
    with pytest.raises(binding.PgError) as e:
        binding.Graph(rp, col)
    assert e.value.code == binding.PG_EINVAL
    # the symmetric closure of the entries, without loops, by definition
    pairs = {(min(v, int(u)), max(v, int(u))) for v in range(g.n) for u in col[rp[v]:rp[v + 1]] if int(u) != v}
    with binding.Graph(rp, col, canonicalize=True) as G:
        n, nnz, dmax = G.info()
        assert (n, nnz) == (g.n, 2 * len(pairs))
        assert nnz == g.col.shape[0] and dmax == int(np.diff(g.row_ptr).max())
        assert [G.cliques(k) for k in (3, 4)] == [oracle.clique_count(g, k) for k in (3, 4)]
        assert [int(x) for x in G.motifs(4)] == [int(x) for x in closed_form.motif4(g)]
    # a clean CSR is unchanged by it; ids or row bounds out of range still fail
    with binding.Graph.from_csr(g, canonicalize=True) as G:
        assert G.info()[1] == g.col.shape[0]
        assert G.cliques(3) == oracle.clique_count(g, 3)
    bad = col.copy()
    bad[0] = g.n
    with pytest.raises(binding.PgError) as e:
        binding.Graph(rp, bad, canonicalize=True)
    assert e.value.code == binding.PG_EINVAL
    with pytest.raises(binding.PgError) as e:
        binding.Graph(np.array([0, 5, 3], np.int64), np.zeros(5, np.int32), canonicalize=True)
    assert e.value.code == binding.PG_EINVAL
