"""Pins of the clique oracle against closed forms, brute force and a
library routine (Pangolin section 2.2: k-clique = k pairwise adjacent
vertices; TC is k = 3)."""
import itertools
from math import comb

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from oracle import brute
from paper_1911_06969_amd import synth


def elem_sym(sizes, k):
    return sum(int(np.prod(c)) for c in itertools.combinations(sizes, k)) if k else 1


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 10])
def test_complete_graph_binomial(n):
    g = synth.complete(n)
    for k in range(1, n + 2):
        assert oracle.clique_count(g, k) == comb(n, k)


def test_empty_graph():
    g = synth.empty(20)
    assert oracle.clique_count(g, 3) == 0
    assert oracle.clique_count(g, 4) == 0
    assert oracle.clique_count(g, 2) == 0


@pytest.mark.parametrize("sizes", [[1, 1, 1], [2, 3], [2, 2, 2], [3, 1, 4, 2], [5, 5, 5, 5]])
def test_complete_multipartite_elementary_symmetric(sizes):
    g = synth.complete_multipartite(sizes)
    for k in range(2, len(sizes) + 2):
        assert oracle.clique_count(g, k) == elem_sym(sizes, k)


def test_disjoint_union_adds():
    a, b = synth.gnp_small(30, 0.4, 1), synth.complete(7)
    u = synth.disjoint_union(a, b)
    for k in (3, 4, 5):
        assert oracle.clique_count(u, k) == oracle.clique_count(a, k) + oracle.clique_count(b, k)


@pytest.mark.parametrize("seed", range(8))
def test_brute_force_small(seed):
    rng = np.random.default_rng(seed)
    g = synth.gnp_small(int(rng.integers(6, 13)), float(rng.uniform(0.2, 0.8)), seed)
    for k in (3, 4, 5):
        assert oracle.clique_count(g, k) == brute.clique_count(g, k)


def test_triangles_trace_cube():
    """TC = trace(A^3)/6, with the sparse product from scipy."""
    g = synth.rmat(12, 8, seed=11)
    A = sp.csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(g.n, g.n))
    tri = int(round((A @ A).multiply(A).sum() / 6))
    assert oracle.clique_count(g, 3) == tri


def test_relabel_invariance():
    g = synth.rmat(11, 8, seed=12)
    perm = np.random.default_rng(3).permutation(g.n)
    h = synth.relabel(g, perm)
    for k in (3, 4, 5):
        assert oracle.clique_count(g, k) == oracle.clique_count(h, k)


def test_roots_partition_total():
    g = synth.rmat(10, 8, seed=13)
    per = oracle.clique_count_roots(g, 4, np.arange(g.n))
    assert int(per.sum()) == oracle.clique_count(g, 4)


def test_edges_and_vertices():
    g = synth.rmat(9, 4, seed=14)
    assert oracle.clique_count(g, 2) == g.n_edges
    assert oracle.clique_count(g, 1) == g.n


# ------------------------------------------------------------ clique listing

@pytest.mark.parametrize("n,k", [(1, 1), (5, 2), (6, 3), (7, 4), (8, 8), (6, 7)])
def test_list_complete_graph_all_subsets(n, k):
    """K_n: the k-cliques are exactly the k-subsets, in lexicographic order."""
    g = synth.complete(n)
    assert oracle.clique_list(g, k) == list(itertools.combinations(range(n), k))


@pytest.mark.parametrize("seed", range(6))
def test_list_matches_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    g = synth.gnp_small(int(rng.integers(5, 12)), float(rng.uniform(0.3, 0.9)), 100 + seed)
    for k in (1, 2, 3, 4, 5):
        assert oracle.clique_list(g, k) == brute.clique_list(g, k)


def test_list_sizes_match_counts():
    """Listing and the C++ clique enumeration agree on R-MAT graphs."""
    g = synth.rmat(9, 8, seed=11)
    for k in (3, 4, 5):
        lst = oracle.clique_list(g, k)
        assert len(lst) == oracle.clique_count(g, k)
        assert len(set(lst)) == len(lst)
        assert all(all(a < b for a, b in zip(t, t[1:])) for t in lst)
