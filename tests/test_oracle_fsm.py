"""Pins of the FSM oracle (edge-subset enumeration + domain support)
against supports computed from injective maps by definition, and against
properties of the minimum-image support (Pangolin section 2.2)."""
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
