"""Pins of the FSM oracle (edge-subset enumeration + domain support)
against supports computed from injective maps by definition, and against
properties of the minimum-image support (Pangolin section 2.2)."""
import itertools

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_1911_06969_amd import synth


def test_pattern_count_sixteen_labels():
    # 136 edges + 16*136 wedges + 816 triangles + 32896 paths + 16*816 stars
    assert oracle.fsm_num_patterns(3, 16) == 49080
    assert oracle.fsm_num_patterns(1, 16) == 136
    assert oracle.fsm_num_patterns(2, 16) == 136 + 16 * 136


@pytest.mark.parametrize("L", [1, 2, 3, 5])
def test_index_matches_enumerated_table(L):
    table = brute.pattern_table(3, L)
    assert len(table) == oracle.fsm_num_patterns(3, L)
    for i, (shape, lab) in enumerate(table):
        assert oracle.fsm_pattern_index(shape, lab, L) == i


def test_index_symmetric_forms():
    L = 16
    assert oracle.fsm_pattern_index(3, [1, 2, 3, 4], L) == oracle.fsm_pattern_index(3, [4, 3, 2, 1], L)
    assert oracle.fsm_pattern_index(4, [1, 9, 2, 5], L) == oracle.fsm_pattern_index(4, [1, 5, 9, 2], L)
    assert oracle.fsm_pattern_index(1, [3, 7, 2], L) == oracle.fsm_pattern_index(1, [3, 2, 7], L)


@pytest.mark.parametrize("seed", range(10))
def test_against_injective_maps(seed):
    rng = np.random.default_rng(200 + seed)
    L = int(rng.integers(1, 4))
    g = synth.gnp_small(int(rng.integers(5, 10)), float(rng.uniform(0.2, 0.6)), seed, n_labels=L)
    want = brute.fsm_supports_all(g, 3)
    got, cnt = oracle.fsm_supports_all(g, 3)
    assert np.array_equal(want, got)
    assert list(cnt) == [brute.edge_subsets(g, j) for j in (1, 2, 3)]


def test_single_label_edge_support_is_non_isolated():
    g = synth.rmat(9, 4, seed=31)
    g.labels = np.zeros(g.n, np.int32)
    g.n_labels = 1
    sup, _ = oracle.fsm_supports_all(g, 1)
    assert int(sup[0]) == int((g.degrees() > 0).sum())


def test_thresholds():
    g = synth.erdos_renyi(400, 0.02, seed=32, n_labels=3)
    allsup, _ = oracle.fsm_supports_all(g, 3)
    assert np.array_equal(oracle.fsm(g, 3, 1), allsup)
    assert not oracle.fsm(g, 3, 10 ** 9).any()
    mid = oracle.fsm(g, 3, 20)
    assert np.array_equal(mid, np.where(allsup >= 20, allsup, 0))


def test_anti_monotone():
    g = synth.erdos_renyi(600, 0.01, seed=33, n_labels=3)
    L = 3
    sup, _ = oracle.fsm_supports_all(g, 3)
    idx = lambda s, lab: oracle.fsm_pattern_index(s, lab, L)
    checked = 0
    for i, (shape, lab) in enumerate(brute.pattern_table(3, L)):
        if sup[i] == 0:
            continue
        if shape == 1:
            c, a, b = lab
            subs = [idx(0, [c, a]), idx(0, [c, b])]
        elif shape == 2:
            a, b, c = lab
            subs = [idx(1, [a, b, c]), idx(1, [b, a, c]), idx(1, [c, a, b])]
        elif shape == 3:
            a, b, c, d = lab
            subs = [idx(1, [b, a, c]), idx(1, [c, b, d])]
        elif shape == 4:
            c, a, b, d = lab
            subs = [idx(1, [c, a, b]), idx(1, [c, a, d]), idx(1, [c, b, d])]
        else:
            continue
        for s in subs:
            assert sup[s] >= sup[i]
            checked += 1
    assert checked > 50


def test_label_renaming():
    L = 3
    g = synth.erdos_renyi(300, 0.02, seed=34, n_labels=L)
    ren = np.array([2, 0, 1], np.int32)
    h = synth.CSR(g.row_ptr, g.col, ren[g.labels], L)
    sg, _ = oracle.fsm_supports_all(g, 3)
    sh, _ = oracle.fsm_supports_all(h, 3)
    for i, (shape, lab) in enumerate(brute.pattern_table(3, L)):
        j = oracle.fsm_pattern_index(shape, [int(ren[x]) for x in lab], L)
        assert sg[i] == sh[j]


# ------------------------------------------------------------ four edges

def _binom(n, k):
    from math import comb
    return comb(n, k) if n >= k >= 0 else 0


@pytest.mark.parametrize("L", [1, 2, 3, 4, 5, 16])
def test_pattern_count_four_edges(L):
    """Block sizes from counting arguments: 5-paths up to reversal
    (palindromes a=e, b=d counted once), 4-stars (centre, multiset of 4
    leaves), forks (centre, multiset of 2 leaves, ordered leg), 4-cycles up
    to the dihedral group (Burnside: identity, two quarter turns, the half
    turn, two reflections through vertices, two through edges), paws
    (degree-3 vertex, pendant, multiset of the other two)."""
    path5 = (L ** 5 + L ** 3) // 2
    star4 = L * _binom(L + 3, 4)
    fork = L * _binom(L + 1, 2) * L * L
    cycle = (L ** 4 + 2 * L + L ** 2 + 2 * L ** 3 + 2 * L ** 2) // 8
    paw = L * L * _binom(L + 1, 2)
    assert (L ** 4 + 2 * L + L ** 2 + 2 * L ** 3 + 2 * L ** 2) % 8 == 0
    assert oracle.fsm_num_patterns(4, L) == oracle.fsm_num_patterns(3, L) + path5 + star4 + fork + cycle + paw


@pytest.mark.parametrize("L", [1, 2, 3])
def test_index_matches_enumerated_table_four_edges(L):
    table = brute.pattern_table(4, L)
    assert len(table) == oracle.fsm_num_patterns(4, L)
    for i, (shape, lab) in enumerate(table):
        assert oracle.fsm_pattern_index(shape, lab, L) == i


def test_index_symmetric_forms_four_edges():
    L = 16
    idx = lambda s, lab: oracle.fsm_pattern_index(s, lab, L)  # noqa: E731
    assert idx(5, [1, 2, 3, 4, 5]) == idx(5, [5, 4, 3, 2, 1])
    assert idx(6, [3, 9, 2, 5, 1]) == idx(6, [3, 1, 2, 5, 9])
    assert idx(7, [3, 9, 2, 5, 1]) == idx(7, [3, 2, 9, 5, 1])
    assert idx(7, [3, 9, 2, 5, 1]) != idx(7, [3, 9, 2, 1, 5])
    cyc = [4, 7, 1, 9]
    for r in range(4):
        rot = cyc[r:] + cyc[:r]
        assert idx(8, rot) == idx(8, cyc) == idx(8, rot[::-1])
    assert idx(8, [1, 2, 1, 3]) != idx(8, [1, 1, 2, 3])
    assert idx(9, [4, 6, 8, 2]) == idx(9, [4, 6, 2, 8])
    assert idx(9, [4, 6, 8, 2]) != idx(9, [6, 4, 8, 2])


@pytest.mark.parametrize("seed", range(8))
def test_against_injective_maps_four_edges(seed):
    rng = np.random.default_rng(700 + seed)
    L = int(rng.integers(1, 4))
    g = synth.gnp_small(int(rng.integers(5, 9)), float(rng.uniform(0.25, 0.6)), seed, n_labels=L)
    want = brute.fsm_supports_all(g, 4)
    got, cnt = oracle.fsm_supports_all(g, 4)
    assert np.array_equal(want, got)
    assert list(cnt) == [brute.edge_subsets(g, j) for j in (1, 2, 3, 4)]


def _one_label(g):
    return synth.CSR(g.row_ptr, g.col, np.zeros(g.n, np.int32), 1)


def test_four_edge_closed_forms_single_label():
    """One label: on the cycle C_n (n >= 5) every 4-edge path lies on the
    cycle (n of them) and every vertex is in every orbit's domain; on the
    path P_n the 5-path's middle position reaches the n - 4 inner vertices;
    K_{1,m} holds C(m, 4) 4-stars, with the centre's domain of size 1;
    K_4 holds three 4-cycles and twelve paws, each position reached by all
    four vertices."""
    L = 1
    idx = lambda s: oracle.fsm_pattern_index(s, [0] * brute.SHAPES[s][0], L)  # noqa: E731
    for n in (5, 6, 9):
        sup, cnt = oracle.fsm_supports_all(_one_label(synth.cycle(n)), 4)
        assert int(cnt[3]) == n
        assert int(sup[idx(5)]) == n and int(sup[idx(8)]) == 0
    for n in (5, 7, 10):
        sup, cnt = oracle.fsm_supports_all(_one_label(synth.path(n)), 4)
        assert int(cnt[3]) == n - 4
        assert int(sup[idx(5)]) == n - 4
    for m in (4, 6, 9):
        sup, cnt = oracle.fsm_supports_all(_one_label(synth.star(m)), 4)
        assert int(cnt[3]) == _binom(m, 4)
        assert int(sup[idx(6)]) == 1
    sup, cnt = oracle.fsm_supports_all(_one_label(synth.complete(4)), 4)
    assert int(cnt[3]) == _binom(6, 4) == 3 + 12
    assert int(sup[idx(8)]) == 4 and int(sup[idx(9)]) == 4


def _identify(edges, labels):
    """(shape, canonical labels) of a connected labelled edge list, by
    matching it against every shape with as many edges and vertices."""
    verts = sorted({x for e in edges for x in e})
    es = {frozenset(e) for e in edges}
    for shape, (nv, sedges) in brute.SHAPES.items():
        if len(sedges) != len(edges) or nv != len(verts):
            continue
        for p in itertools.permutations(verts):
            if {frozenset((p[a], p[b])) for a, b in sedges} == es:
                return shape, brute.canonical_labels(shape, [labels[p[i]] for i in range(nv)])
    raise AssertionError("no shape")


def test_anti_monotone_four_edges():
    """A 4-edge pattern's support is at most that of each connected 3-edge
    pattern it contains."""
    L = 2
    g = synth.erdos_renyi(300, 0.012, seed=35, n_labels=L)
    sup, _ = oracle.fsm_supports_all(g, 4)
    checked = 0
    for i, (shape, lab) in enumerate(brute.pattern_table(4, L)):
        if brute.SHAPE_EDGES[shape] != 4 or sup[i] == 0:
            continue
        edges = brute.SHAPES[shape][1]
        for drop in range(4):
            rest = [e for j, e in enumerate(edges) if j != drop]
            vs = {x for e in rest for x in e}
            comp = {rest[0][0]}
            for _ in range(4):
                comp |= {x for e in rest if comp & set(e) for x in e}
            if comp != vs:
                continue
            s3, l3 = _identify(rest, lab)
            assert sup[oracle.fsm_pattern_index(s3, l3, L)] >= sup[i]
            checked += 1
    assert checked > 100


def test_label_renaming_four_edges():
    L = 3
    g = synth.erdos_renyi(200, 0.02, seed=36, n_labels=L)
    ren = np.array([1, 2, 0], np.int32)
    h = synth.CSR(g.row_ptr, g.col, ren[g.labels], L)
    sg, _ = oracle.fsm_supports_all(g, 4)
    sh, _ = oracle.fsm_supports_all(h, 4)
    for i, (shape, lab) in enumerate(brute.pattern_table(4, L)):
        j = oracle.fsm_pattern_index(shape, [int(ren[x]) for x in lab], L)
        assert sg[i] == sh[j]
