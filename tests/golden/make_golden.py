"""Writes full_configs.json: oracle results on the full-size synthetic
workloads.  Calls only the seeded generators and oracle/ (never the HIP
library).  Run from the repository root:

    python tests/golden/make_golden.py [section ...]

Sections: triangle_rmat_s14, clique_rmat_s21, motif_rmat_s18, fsm_er_500k,
motif_batch_100k, and rmat_sweep_s20 .. rmat_sweep_s25 (the weak-scaling
graphs: R-MAT with edge factor 10, seed 7; triangles at every scale,
4-cliques up to scale 23).
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import closed_form  # noqa: E402
from paper_1911_06969_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_configs.json")


def sec_triangle():
    g = synth.triangle_rmat()
    return {"n": g.n, "edges": g.n_edges, "k3": oracle.clique_count(g, 3), "k4": oracle.clique_count(g, 4),
            "motif3": [int(x) for x in closed_form.motif3(g)],
            "motif4": [int(x) for x in closed_form.motif4(g)]}


def sec_clique(ks=(3, 4)):
    g = synth.clique_rmat()
    out = {"n": g.n, "edges": g.n_edges}
    for k in ks:
        t = time.time()
        out[f"k{k}"] = oracle.clique_count(g, k)
        print(f"clique k={k}: {out[f'k{k}']} in {time.time() - t:.1f}s", flush=True)
    return out


def sec_motif():
    g = synth.motif_rmat()
    return {"n": g.n, "edges": g.n_edges, "motif3": [int(x) for x in closed_form.motif3(g)],
            "motif4": [int(x) for x in closed_form.motif4(g)]}


def sec_fsm():
    g = synth.fsm_er()
    sup, cnt = oracle.fsm_supports_all(g, 3)
    out = {"n": g.n, "edges": g.n_edges, "embeddings": [int(x) for x in cnt]}
    for sigma in (1000,):
        f = np.where(sup >= sigma, sup, 0).astype(np.uint64)
        nz = np.nonzero(f)[0]
        out[f"sigma{sigma}"] = {
            "n_frequent": int(nz.shape[0]),
            "sha256": hashlib.sha256(f.tobytes()).hexdigest(),
            "sum": int(f.sum()),
            "sample_index": [int(i) for i in nz[:: max(1, nz.shape[0] // 200)]],
            "sample_support": [int(f[i]) for i in nz[:: max(1, nz.shape[0] // 200)]],
        }
    return out


def sec_sweep(scale):
    """The weak-scaling sweep's graph of 2^scale vertices (edge factor 10,
    seed 7): triangles, and 4-cliques up to scale 23."""
    def run():
        t = time.time()
        g = synth.rmat(scale, 10, seed=7)
        out = {"n": g.n, "edges": g.n_edges}
        print(f"sweep scale {scale}: graph in {time.time() - t:.1f}s", flush=True)
        ks = (3, 4) if scale <= 23 else (3,)
        for k in ks:
            t = time.time()
            out[f"k{k}"] = oracle.clique_count(g, k)
            print(f"sweep scale {scale} k={k}: {out[f'k{k}']} in {time.time() - t:.1f}s", flush=True)
        return out
    return run


_BATCH = None


def _batch_rows(rng_slice):
    lo, hi = rng_slice
    return np.stack([closed_form.motif4(_BATCH.graph(i), nthreads=1) for i in range(lo, hi)]).astype(np.uint64)


def sec_batch():
    import multiprocessing as mp
    global _BATCH
    _BATCH = synth.motif_batch()
    G = _BATCH.n_graphs
    step = 500
    slices = [(i, min(G, i + step)) for i in range(0, G, step)]
    with mp.get_context("fork").Pool(max(1, os.cpu_count() or 1)) as pool:
        rows = np.concatenate(pool.map(_batch_rows, slices))
    idx = list(range(0, G, 997))
    return {"n_graphs": G, "sum": [int(x) for x in rows.sum(axis=0)],
            "sha256": hashlib.sha256(rows.tobytes()).hexdigest(),
            "sample_index": idx, "sample_rows": [[int(x) for x in rows[i]] for i in idx]}


SECTIONS = {
    "motif_batch_100k": sec_batch,
    "triangle_rmat_s14": sec_triangle,
    "clique_rmat_s21": sec_clique,
    "clique_rmat_s21_k5": lambda: sec_clique((5,)),
    "motif_rmat_s18": sec_motif,
    "fsm_er_500k": sec_fsm,
}
for _sc in range(20, 26):
    SECTIONS[f"rmat_sweep_s{_sc}"] = sec_sweep(_sc)


def main(names):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    # the sweep sections are written only when named (hours of CPU at the top scales)
    for name in names or [n for n in SECTIONS if not n.startswith("rmat_sweep")]:
        t = time.time()
        data[name] = SECTIONS[name]()
        print(name, f"{time.time() - t:.1f}s", flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:])
