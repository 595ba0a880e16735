"""Closed-form motif counts -- TEST INFRASTRUCTURE ONLY.

Every connected 4-vertex pattern H occurs a fixed number of times as a
spanning (non-induced) subgraph of every other 4-vertex pattern; so the
non-induced counts N_H, which have simple formulas, are a triangular linear
combination of the induced counts I_P the motif-counting method returns
(Pangolin section 2.2 notes such relations between pattern counts).

Non-induced counts (T = triangles, t_v = triangles at v, t_e = triangles on
edge e, c(u,w) = common neighbours of u and w):
  N_star    = sum_v C(d_v, 3)
  N_path    = sum_{uv in E} (d_u - 1)(d_v - 1) - 3T
  N_cycle   = (1/2) sum_{u<w} C(c(u,w), 2)
  N_paw     = sum_v t_v (d_v - 2)
  N_diamond = sum_e C(t_e, 2)
  N_clique  = number of 4-cliques
Copies of each pattern inside the others (rows: counted pattern):
  star:    star 1, paw 1, diamond 2, clique 4
  path:    path 1, cycle 4, paw 2, diamond 6, clique 12
  cycle:   cycle 1, diamond 1, clique 3
  paw:     paw 1, diamond 4, clique 12
  diamond: diamond 1, clique 6
which is inverted by back-substitution below.  3-motifs: wedges induced =
sum_v C(d_v, 2) - 3T, triangles = T.
"""
from __future__ import annotations

import numpy as np

from . import clique_count, motif_parts


def motif3(g, nthreads: int = 0) -> np.ndarray:
    p = motif_parts(g, nthreads)
    T = p["triangles"]
    return np.array([p["wedges_noninduced"] - 3 * T, T], dtype=np.uint64)


def motif4(g, nthreads: int = 0) -> np.ndarray:
    p = motif_parts(g, nthreads)
    T = p["triangles"]
    n_star = p["stars_noninduced"]
    n_path = p["p4_raw"] - 3 * T
    assert p["c4_twice"] % 2 == 0
    n_cycle = p["c4_twice"] // 2
    n_paw = p["paws_noninduced"]
    n_dia = p["diamonds_noninduced"]
    n_k4 = clique_count(g, 4, nthreads)
    i_k4 = n_k4
    i_dia = n_dia - 6 * i_k4
    i_paw = n_paw - 4 * i_dia - 12 * i_k4
    i_cycle = n_cycle - i_dia - 3 * i_k4
    i_path = n_path - 2 * i_paw - 4 * i_cycle - 6 * i_dia - 12 * i_k4
    i_star = n_star - i_paw - 2 * i_dia - 4 * i_k4
    vals = [i_path, i_star, i_cycle, i_paw, i_dia, i_k4]
    assert all(v >= 0 for v in vals), vals
    return np.array(vals, dtype=np.uint64)
