"""Brute-force oracle for tiny graphs -- TEST INFRASTRUCTURE ONLY.

Everything here follows a definition directly, with no pruning:
  * k-cliques: every k-subset, pairwise adjacent (Pangolin section 2.2).
  * k-motifs: every k-subset whose induced subgraph is connected, grouped by
    isomorphism class (sections 2.1-2.2, vertex-induced embeddings); for
    k = 5 the class is the smallest relabelled adjacency mask.
  * FSM: for each labelled pattern with at most 4 edges, every injective,
    label-preserving map of its vertices into the graph that sends pattern
    edges to graph edges; the minimum-image (domain) support is the smallest
    number of distinct images over the pattern's vertices (section 2.2).
Use on graphs of about a dozen vertices.
"""
from __future__ import annotations

import itertools

import numpy as np


def dense_adj(g) -> np.ndarray:
    A = np.zeros((g.n, g.n), dtype=bool)
    for v in range(g.n):
        A[v, g.adj(v)] = True
    return A


def clique_count(g, k: int) -> int:
    A = dense_adj(g)
    total = 0
    for s in itertools.combinations(range(g.n), k):
        if all(A[a, b] for a, b in itertools.combinations(s, 2)):
            total += 1
    return total


def clique_list(g, k: int) -> list:
    """Every k-clique as its ascending tuple of vertex ids, in lexicographic
    order (all k-subsets, kept when pairwise adjacent)."""
    A = dense_adj(g)
    return [s for s in itertools.combinations(range(g.n), k)
            if all(A[a, b] for a, b in itertools.combinations(s, 2))]


def _connected(A, s) -> bool:
    s = list(s)
    seen = {s[0]}
    stack = [s[0]]
    while stack:
        x = stack.pop()
        for y in s:
            if y not in seen and A[x, y]:
                seen.add(y)
                stack.append(y)
    return len(seen) == len(s)


def motif_class(A, s) -> int:
    """Isomorphism class of a connected induced subgraph on 3 or 4 vertices,
    from its edge count and largest degree:
      3 vertices: 0 wedge, 1 triangle
      4 vertices: 0 path, 1 star, 2 cycle, 3 paw (tailed triangle),
                  4 diamond, 5 clique."""
    deg = [sum(1 for y in s if y != x and A[x, y]) for x in s]
    e = sum(deg) // 2
    if len(s) == 3:
        return 1 if e == 3 else 0
    if e == 3:
        return 1 if max(deg) == 3 else 0
    if e == 4:
        return 3 if max(deg) == 3 else 2
    return 4 if e == 5 else 5


# Five vertices: the 21 connected graphs, numbered by (number of edges,
# canonical code).  A graph on positions 0..4 is a 10-bit mask, bit
# b(b-1)/2 + a for the pair a < b (the 4-vertex pair order extended by
# 04, 14, 24, 34); its canonical code is the smallest mask over the 120
# relabellings of the positions.
PAIRS5 = [(a, b) for b in range(5) for a in range(b)]


def _relabel5(m: int, perm) -> int:
    out = 0
    for i, (a, b) in enumerate(PAIRS5):
        if (m >> i) & 1:
            x, y = sorted((perm[a], perm[b]))
            out |= 1 << (y * (y - 1) // 2 + x)
    return out


def _mask_connected5(m: int) -> bool:
    seen, stack = {0}, [0]
    while stack:
        x = stack.pop()
        for i, (a, b) in enumerate(PAIRS5):
            if (m >> i) & 1 and x in (a, b):
                y = b if x == a else a
                if y not in seen:
                    seen.add(y)
                    stack.append(y)
    return len(seen) == 5


def motif5_classes() -> list:
    """Canonical codes of the connected 5-vertex graphs, in class order."""
    perms = list(itertools.permutations(range(5)))
    codes = {min(_relabel5(m, p) for p in perms) for m in range(1 << 10) if _mask_connected5(m)}
    return sorted(codes, key=lambda c: (bin(c).count("1"), c))


_CLASS5 = None


def motif5_class_of_mask() -> dict:
    """10-bit mask -> class id, for the connected masks."""
    global _CLASS5
    if _CLASS5 is None:
        perms = list(itertools.permutations(range(5)))
        index = {c: i for i, c in enumerate(motif5_classes())}
        _CLASS5 = {m: index[min(_relabel5(m, p) for p in perms)]
                   for m in range(1 << 10) if _mask_connected5(m)}
    return _CLASS5


def motif_counts(g, k: int) -> np.ndarray:
    A = dense_adj(g)
    if k == 5:
        cls = motif5_class_of_mask()
        out = np.zeros(21, dtype=np.uint64)
        for s in itertools.combinations(range(g.n), 5):
            m = 0
            for i, (a, b) in enumerate(PAIRS5):
                if A[s[a], s[b]]:
                    m |= 1 << i
            c = cls.get(m)
            if c is not None:
                out[c] += 1
        return out
    out = np.zeros(2 if k == 3 else 6, dtype=np.uint64)
    for s in itertools.combinations(range(g.n), k):
        if _connected(A, s):
            out[motif_class(A, s)] += 1
    return out


def connected_subsets(g, k: int) -> int:
    A = dense_adj(g)
    return sum(1 for s in itertools.combinations(range(g.n), k) if _connected(A, s))


# --------------------------------------------------------------------- FSM

# shape id -> (number of vertices, edges between pattern vertex positions)
SHAPES = {
    0: (2, [(0, 1)]),                            # single edge, labels (a, b)
    1: (3, [(0, 1), (0, 2)]),                    # wedge, labels (centre, leaf, leaf)
    2: (3, [(0, 1), (0, 2), (1, 2)]),            # triangle
    3: (4, [(0, 1), (1, 2), (2, 3)]),            # path on 4 vertices, labels along the path
    4: (4, [(0, 1), (0, 2), (0, 3)]),            # 3-star, labels (centre, leaves)
    5: (5, [(0, 1), (1, 2), (2, 3), (3, 4)]),    # path on 5 vertices
    6: (5, [(0, 1), (0, 2), (0, 3), (0, 4)]),    # 4-star
    7: (5, [(0, 1), (0, 2), (0, 3), (3, 4)]),    # fork: centre, two leaves, leg (middle, end)
    8: (4, [(0, 1), (1, 2), (2, 3), (3, 0)]),    # 4-cycle, labels around the cycle
    9: (4, [(0, 1), (0, 2), (0, 3), (2, 3)]),    # paw: degree-3 vertex, pendant, the two others
}
SHAPE_EDGES = {s: len(e) for s, (_, e) in SHAPES.items()}


def _automorphisms(shape: int) -> list:
    """Position permutations that map the shape's edge set onto itself."""
    nv, edges = SHAPES[shape]
    es = {frozenset(e) for e in edges}
    return [p for p in itertools.permutations(range(nv))
            if {frozenset((p[a], p[b])) for a, b in edges} == es]


def canonical_labels(shape: int, labels) -> tuple:
    """Representative label tuple of a labelled shape: the smallest tuple
    over the shape's automorphisms (a label tuple read through each)."""
    lab = tuple(labels)
    return min(tuple(lab[p[i]] for i in range(len(lab))) for p in _automorphisms(shape))


def pattern_table(max_edges: int, L: int):
    """The dense pattern numbering, block by block in shape order (edge,
    wedge, triangle, 4-path, 3-star, 5-path, 4-star, fork, 4-cycle, paw);
    within a block the representative label tuples (canonical_labels) in
    lexicographic order.  Returns a list of (shape, labels) whose position is
    the index."""
    table = []
    for shape in sorted(SHAPES):
        if SHAPE_EDGES[shape] > max_edges:
            continue
        nv = SHAPES[shape][0]
        autos = _automorphisms(shape)
        for t in itertools.product(range(L), repeat=nv):
            if all(tuple(t[p[i]] for i in range(nv)) >= t for p in autos):
                table.append((shape, t))
    return table


def pattern_index(shape: int, labels, L: int, max_edges: int = 3) -> int:
    table = pattern_table(max(max_edges, SHAPE_EDGES[shape]), L)
    return table.index((shape, canonical_labels(shape, labels)))


def mni_support(g, shape: int, labels) -> int:
    """Minimum-image support of one labelled pattern, by enumerating every
    injective label-preserving edge-preserving map."""
    A = dense_adj(g)
    nv, pedges = SHAPES[shape]
    dom = [set() for _ in range(nv)]
    cands = [[v for v in range(g.n) if g.labels[v] == labels[i]] for i in range(nv)]
    for phi in itertools.product(*cands):
        if len(set(phi)) < nv:
            continue
        if all(A[phi[a], phi[b]] for a, b in pedges):
            for i in range(nv):
                dom[i].add(phi[i])
    return min(len(d) for d in dom)


def fsm_supports_all(g, max_edges: int) -> np.ndarray:
    """Unfiltered supports at the dense index."""
    table = pattern_table(max_edges, g.n_labels)
    out = np.zeros(len(table), dtype=np.uint64)
    present = set(int(x) for x in g.labels)
    for i, (shape, lab) in enumerate(table):
        if all(x in present for x in lab):
            out[i] = mni_support(g, shape, lab)
    return out


def fsm(g, max_edges: int, min_support: int) -> np.ndarray:
    sup = fsm_supports_all(g, max_edges)
    sup[sup < np.uint64(max(min_support, 0))] = 0
    return sup


def edge_subsets(g, j: int) -> int:
    """Number of connected j-edge subsets (edge-induced embeddings)."""
    E = [tuple(e) for e in g.edges()]
    total = 0
    for s in itertools.combinations(E, j):
        verts = {x for e in s for x in e}
        # connectivity of the edge set
        comp = {next(iter(verts))}
        changed = True
        while changed:
            changed = False
            for a, b in s:
                if (a in comp) != (b in comp):
                    comp |= {a, b}
                    changed = True
        if comp == verts:
            total += 1
    return total
