"""Benchmark: k-clique counting on the R-MAT scale-21 graph (one GPU).

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload clique4]
python bench.py --workload rmat-sweep [--sweep-scales 20,21,22,23,24,25]

One step = one pass of the clique hot path over the resident graph:
pg_count_cliques(g, 4) = level-1 count pass, scan, write of the triangle
level, and the fused last level.  The graph and its degree-ordered DAG are
device resident before timing starts (preprocessing and host-to-device
copies are excluded, as in the paper's evaluation).

Prints one JSON line.  `preprocess` gives the graph load and the first call
(which also builds the DAG), both outside the timed steps.  `roofline` is for
the dominant kernel (the one
with the most time per step among the kernels that record their algorithmic
bytes), from HIP events recorded around every launch during the timed
steps; `cpu_baseline` times the CPU oracle on a bounded sample of the same
workload (rank 0, N = 1 only).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "embeddings/s, 4-clique & 4-motif on RMAT; batched graphs/s vs plain, p99 latency"
HBM_PEAK_GBS = 8000.0


def note(*msg):
    """Progress of the run, on stderr (stdout carries only the JSON line)."""
    print("[bench]", *msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="clique4",
                    choices=["clique4", "clique5", "motif4", "motif3", "motif5", "tc", "fsm", "copy", "tune-batch",
                             "rmat-sweep", "serve"],
                    help="copy: a plain 1 GiB device-to-device copy, the known-size reference "
                         "for scaling HBM counters; rmat-sweep: triangles and 4-cliques on R-MAT "
                         "graphs of 2^20 .. 2^25 vertices, average degree 20 (weak scaling)")
    ap.add_argument("--sweep-scales", default="20,21,22,23,24,25")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the 4-motif, batched and served measurements")
    ap.add_argument("--plain-sample", type=int, default=2000)
    ap.add_argument("--serve-requests", type=int, default=200000)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-batch", type=int, default=1024)
    ap.add_argument("--cpu-sample-seconds", type=float, default=15.0)
    ap.add_argument("--tuning", default=os.path.join(ROOT, "profiles", "batch_tuning.json"),
                    help="batch-kernel parameters picked by the autotuner (applied when present)")
    ap.add_argument("--tuning-out", default=os.path.join(ROOT, "profiles", "batch_tuning.json"),
                    help="where --workload tune-batch writes its result")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="measured HBM bytes per launch of the dominant kernel (from rocprofv3 --pmc)")
    return ap.parse_args()


def cpu_baseline_cliques(g, k, want_seconds):
    """Oracle (unchanged) on a random sample of roots: the cliques whose first
    vertex in the degree order is a sampled vertex."""
    import numpy as np

    import oracle
    rng = np.random.default_rng(12345)
    n = g.n
    # calibrate: a call's fixed cost (its own degree ordering) and the
    # marginal cost of 1% of the roots; then size the sample to ~want_seconds
    t = time.perf_counter()
    oracle.clique_count_roots(g, k, rng.choice(n, 1))
    fixed = time.perf_counter() - t
    frac = 0.01
    roots = np.sort(rng.choice(n, max(1, int(n * frac)), replace=False))
    t = time.perf_counter()
    oracle.clique_count_roots(g, k, roots)
    marginal = max(time.perf_counter() - t - fixed, 1e-3)
    frac = min(1.0, frac * max(want_seconds - fixed, 1.0) / marginal)
    roots = np.sort(rng.choice(n, max(1, int(n * frac)), replace=False))
    t = time.perf_counter()
    per = oracle.clique_count_roots(g, k, roots)
    dt = time.perf_counter() - t
    found = int(per.sum())
    return {
        "value": found / dt,
        "unit": "embeddings/s",
        "cores": oracle.max_threads(),
        "kind": "oracle",
        "sample": f"{roots.shape[0]} random root vertices ({100 * frac:.2f}% of {n}); "
                  f"{found} {k}-cliques whose first vertex in the degree order is a root, in {dt:.1f} s",
    }


def cpu_baseline_motifs(g, k):
    """The oracle's closed form on the whole graph: non-induced counts from
    degrees, triangles, common neighbours and 4-cliques, then the
    triangular inversion to induced counts.  (The oracle's ESU enumeration
    is orders of magnitude slower here: it copies extension sets, and near
    the scale-18 hubs one root can take minutes.)"""
    from oracle import closed_form, max_threads
    t = time.perf_counter()
    c = closed_form.motif4(g) if k == 4 else closed_form.motif3(g)
    dt = time.perf_counter() - t
    found = int(c.sum())
    return {
        "value": found / dt,
        "unit": "embeddings/s",
        "cores": max_threads(),
        "kind": "oracle",
        "sample": f"the whole graph by the oracle's closed form ({found} {k}-motif embeddings in {dt:.1f} s)",
    }


def cpu_baseline_motif5(g, want_seconds: float = 10.0):
    """The oracle's ESU over a random sample of roots (5-sets whose smallest
    vertex is a root), grown until it takes about want_seconds."""
    import numpy as np
    from oracle import max_threads, motif_esu_roots
    rng = np.random.default_rng(13)
    perm = rng.permutation(g.n).astype(np.int64)
    take, dt, found = 256, 0.0, 0
    while True:
        roots = np.sort(perm[:take])
        t = time.perf_counter()
        found = int(motif_esu_roots(g, 5, roots).sum())
        dt = time.perf_counter() - t
        if dt >= want_seconds / 4 or take >= g.n:
            break
        take = min(g.n, take * 4)
    return {
        "value": found / dt,
        "unit": "embeddings/s",
        "cores": max_threads(),
        "kind": "oracle",
        "sample": f"{take} random root vertices of {g.n}: {found} 5-motif embeddings whose smallest vertex "
                  f"is a root, ESU in {dt:.1f} s",
    }


def cpu_baseline_fsm(n_sample: int = 200_000):
    """The oracle's edge-subset enumeration with domain sets, patterns of up
    to 3 edges, unfiltered, on a smaller graph of the same recipe (labelled
    G(n, p) with average degree 8 and 16 labels): domain supports do not
    split over parts of a graph, so the sample is a whole graph of n_sample
    vertices.  The embeddings it enumerates are the unit."""
    from oracle import fsm_supports_all, max_threads
    from paper_1911_06969_amd import synth
    g = synth.erdos_renyi(n_sample, 8.0 / (n_sample - 1), seed=4, n_labels=16)
    t = time.perf_counter()
    _, cnt = fsm_supports_all(g, 3)
    dt = time.perf_counter() - t
    found = int(cnt.sum())
    return {
        "value": found / dt,
        "unit": "embeddings/s",
        "cores": max_threads(),
        "kind": "oracle",
        "sample": f"labelled G(n,p) n={n_sample}, average degree 8, 16 labels, seed 4 (the workload's recipe at "
                  f"{100 * n_sample / 500000:.0f}% of its vertices): {found} embeddings of 1-3 edges with domain "
                  f"sets in {dt:.1f} s",
    }


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the design for sharding is described in DESIGN.md). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1911_06969_amd import binding, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()

    w = args.workload
    if w == "copy":
        nbytes = 1 << 30
        a = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda").fill_(1)
        b = torch.empty_like(a)
        for _ in range(args.warmup):
            b.copy_(a)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        print(json.dumps({"workload": "copy", "bytes_read": nbytes, "bytes_written": nbytes,
                          "ms_per_copy": 1000 * dt, "GBps_read_plus_write": 2 * nbytes / dt / 1e9}), flush=True)
        return
    if w == "tune-batch":
        from paper_1911_06969_amd import tune
        b = synth.motif_batch()
        h = binding.pg_batch_load(b.voff, b.row_ptr, b.col)
        rng = np.random.default_rng(9)
        ids = np.sort(rng.choice(b.n_graphs, 20000, replace=False))
        n_cu = torch.cuda.get_device_properties(0).multi_processor_count
        best, table = tune.tune(h, ids, n_cu, log=lambda r: print(json.dumps(r), flush=True))
        binding.pg_batch_free(h)
        out = args.tuning_out
        os.makedirs(os.path.dirname(out), exist_ok=True)
        tune.save(out, best, table, "sample: 20,000 of the 100,000 graphs of the motif batch (seed 9), "
                                    "command: python bench.py --workload tune-batch")
        print(json.dumps({"best": best}), flush=True)
        return
    if w == "rmat-sweep":
        rmat_sweep(args, binding, synth, stream)
        return
    if w == "serve":
        print(json.dumps({"workload": "serve", "batch": measure_batch_and_serve(args)}), flush=True)
        return
    line = measure(w, args, args.steps, args.warmup, not args.no_cpu_baseline, stream)
    secondary = {}
    if w == "clique4" and not args.no_secondary:
        for sw, steps in (("motif4", 2), ("clique5", 3), ("tc", 20), ("motif3", 5), ("fsm", 3)):
            note("secondary:", sw)
            sec = measure(sw, args, steps, 1, not args.no_cpu_baseline, stream)
            secondary[sw] = {k: sec[k] for k in ("config", "value", "unit", "ms_per_step", "steps", "result",
                                                 "roofline", "cpu_baseline", "kernels") if k in sec}
        note("secondary: batched graphs, plain sample, serving")
        secondary["batch"] = measure_batch_and_serve(args)
    out = {
        "metric": METRIC,
        "value": line["value"],
        "unit": line["unit"],
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": line["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": line["data"],
        "config": line["config"],
        "result": line["result"],
        "roofline": line["roofline"],
        "cpu_baseline": line["cpu_baseline"],
        "preprocess": line["preprocess"],
        "kernels": line["kernels"],
        "secondary": secondary or None,
    }
    print(json.dumps(out), flush=True)


def workload_of(w, synth):
    """(graph, one step, description) of a named workload."""
    if w == "fsm":
        g = synth.fsm_er()
        return g, (lambda G: G.fsm(3, 1000)[1]), {
            "workload": "frequent subgraph mining up to 3 edges, sigma 1000, labelled G(n,p) n=500,000, "
                        "average degree 8, 16 labels, seed 4", "vertices": g.n, "edges": g.n_edges}
    if w in ("clique4", "clique5"):
        g = synth.clique_rmat()
        k = 4 if w == "clique4" else 5
        return g, (lambda G: G.cliques(k)), {
            "workload": f"{k}-clique counting, R-MAT scale 21 (2,097,152 vertices), edge factor 13, "
                        f"a=0.57 b=0.19 c=0.19, degree-ordered DAG, int32 CSR, seed 2",
            "k": k, "vertices": g.n, "edges": g.n_edges}
    if w == "motif5":
        n = 100_000
        g = synth.erdos_renyi(n, 8.0 / (n - 1), seed=12)
        return g, (lambda G: G.motifs(5)), {"workload": "5-motif counting, G(n,p) n=100,000, average degree 8, "
                                                        "seed 12", "k": 5, "vertices": g.n, "edges": g.n_edges}
    if w == "tc":
        g = synth.triangle_rmat()
        return g, (lambda G: G.cliques(3)), {"workload": "triangle counting, R-MAT scale 14, edge factor 8, seed 1",
                                             "k": 3, "vertices": g.n, "edges": g.n_edges}
    g = synth.motif_rmat()
    k = 4 if w == "motif4" else 3
    return g, (lambda G: G.motifs(k)), {
        "workload": f"{k}-motif counting, R-MAT scale 18 (262,144 vertices), edge factor 8, undirected int32 CSR, "
                    f"seed 3", "k": k, "vertices": g.n, "edges": g.n_edges}


def measure(w, args, steps, warmup, cpu_leg, stream):
    """Times `steps` steps of workload w on the resident graph, with the
    dominant kernel's roofline from HIP events and, when asked, the oracle
    on a bounded sample of the same workload."""
    import numpy as np
    import torch

    from paper_1911_06969_amd import binding, synth
    g, run, workload = workload_of(w, synth)
    k = workload.get("k")

    note("workload", w, "graph ready:", g.n, "vertices")
    # preprocessing, excluded from the timed steps and reported beside them:
    # the load (host-to-device copy, validation) and the first call, which
    # also builds the degree-ordered DAG (and, for cliques, the mask plan)
    torch.cuda.synchronize()
    t_load = time.perf_counter()
    G = binding.Graph.from_csr(g, stream=stream)
    torch.cuda.synchronize()
    t_first = time.perf_counter()
    result = None
    for i in range(warmup):
        result = run(G)
        if i == 0:
            torch.cuda.synchronize()
            t_first_end = time.perf_counter()
    torch.cuda.synchronize()
    preprocess = {"load_ms": round(1000 * (t_first - t_load), 2)}
    if warmup > 0:
        preprocess["first_call_ms"] = round(1000 * (t_first_end - t_first), 2)
    note("warm-up done")

    binding.pg_profile_reset()
    binding.pg_profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        result = run(G)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    binding.pg_profile_enable(False)
    note(f"{w}: timed {steps} steps in {elapsed:.3f} s")

    found = int(np.sum(result)) if not isinstance(result, int) else result
    if w == "fsm":
        # embeddings generated per step (all levels); result = frequent patterns
        emb = binding.pg_profile_query("fsm_embeddings")
        workload["frequent_patterns"] = result
        found = int(emb[2] / steps) if emb else 0
    ms_per_step = 1000.0 * elapsed / steps
    value = found * steps / elapsed

    roofline = None
    kernels = {}
    for name in binding.pg_profile_list():
        q = binding.pg_profile_query(name)
        if q and not name.endswith("_work"):
            kernels[name] = {"ms_per_step": q[0] / steps, "launches_per_step": q[1] / steps}
    # the dominant kernel is the one with the largest time per step that
    # records its algorithmic bytes
    with_work = [n for n in kernels if binding.pg_profile_query(n + "_work")]
    if with_work:
        dominant = max(with_work, key=lambda n: kernels[n]["ms_per_step"])
        prof = binding.pg_profile_query(dominant)
        work = binding.pg_profile_query(dominant + "_work")
        if prof and work and prof[1] > 0:
            avg_s = prof[0] / 1000.0 / prof[1]
            bytes_per_launch = work[2] / prof[1]
            achieved = bytes_per_launch / avg_s / 1e9
            traffic = None
            if os.path.exists(args.traffic):
                with open(args.traffic) as f:
                    t = json.load(f)
                entry = t.get(w)
                if entry and entry.get("kernel") == dominant and entry.get("kernel_source_sha") == kernel_source_sha(w):
                    traffic = entry["bytes_per_launch"]
            roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                        "kernel": dominant, "avg_launch_ms": round(1000 * avg_s, 3),
                        "algorithmic_bytes_per_launch": bytes_per_launch}

    cpu = None
    if cpu_leg:
        note("cpu baseline (oracle)", w)
        if w.startswith("clique") or w == "tc":
            cpu = cpu_baseline_cliques(g, k, args.cpu_sample_seconds)
        elif w == "motif5":
            cpu = cpu_baseline_motif5(g, args.cpu_sample_seconds)
        elif w.startswith("motif"):
            cpu = cpu_baseline_motifs(g, k)
        elif w == "fsm":
            cpu = cpu_baseline_fsm()
    G.close()
    return {
        "config": workload, "value": value, "unit": "embeddings/s", "ms_per_step": ms_per_step, "steps": steps,
        "result": found if isinstance(result, int) else [int(x) for x in result],
        "data": "synthetic (seeded G(n,p))" if w in ("fsm", "motif5") else "synthetic (seeded R-MAT)",
        "roofline": roofline, "cpu_baseline": cpu, "preprocess": preprocess, "kernels": kernels,
    }


def rmat_sweep(args, binding, synth, stream):
    """Weak scaling as in the paper's R-MAT experiment: graphs of 2^s vertices
    and average degree 20 (edge factor 10, a=0.57 b=0.19 c=0.19, seed 7), and
    per graph the time of one triangle count and one 4-clique count after a
    warm-up call, normalised to the smallest graph."""
    import torch
    rows = []
    for sc in [int(x) for x in args.sweep_scales.split(",") if x]:
        t0 = time.perf_counter()
        g = synth.rmat(sc, 10, seed=7)
        note(f"scale {sc}: {g.n} vertices, {g.n_edges} edges, generated in {time.perf_counter() - t0:.1f} s")
        row = {"scale": sc, "vertices": g.n, "edges": g.n_edges}
        with binding.Graph.from_csr(g, stream=stream) as G:
            for k, key in ((3, "tc"), (4, "cf4")):
                G.cliques(k)   # warm-up (builds the DAG on the first call)
                torch.cuda.synchronize()
                t = time.perf_counter()
                c = G.cliques(k)
                torch.cuda.synchronize()
                ms = 1000 * (time.perf_counter() - t)
                row[key + "_ms"] = round(ms, 3)
                row[key + "_count"] = int(c)
                note(f"scale {sc}: {k}-cliques {c} in {ms:.1f} ms")
        rows.append(row)
        del g
    base = rows[0] if rows else None
    for r in rows:
        for key in ("tc", "cf4"):
            r[key + "_vs_first"] = round(r[key + "_ms"] / base[key + "_ms"], 3) if base[key + "_ms"] > 0 else None
    print(json.dumps({"workload": "R-MAT weak-scaling sweep: triangles and 4-cliques, edge factor 10 "
                                  "(average degree 20), a=0.57 b=0.19 c=0.19, seed 7",
                      "data": "synthetic (seeded R-MAT)", "rows": rows}), flush=True)


def measure_batch_and_serve(args):
    """Batched 4-motif counting of 100,000 small G(n, p) graphs in one
    persistent launch, the plain one-graph-per-launch path on a sample of the
    same graphs, and the serving loop at three offered loads."""
    import numpy as np
    import torch

    from paper_1911_06969_amd import binding, serve, synth
    out = {"workload": "4-motif counting of 100,000 G(n,p), n~U{10..400}, p~U[0.02,0.3], seed 5"}
    b = synth.motif_batch()
    h = binding.pg_batch_load(b.voff, b.row_ptr, b.col)
    try:
        tuned = args.tuning
        if tuned and os.path.exists(tuned):
            from paper_1911_06969_amd import tune
            best = tune.load(tuned)
            binding.pg_batch_set_params(h, best["block_threads"], best["split_work"], best["grid_blocks"])
            out["params"] = best
        counts = binding.pg_batch_count_motifs(h, 4, None, n_graphs=b.n_graphs)   # warm-up
        torch.cuda.synchronize()
        reps = 3
        t = time.perf_counter()
        for _ in range(reps):
            counts = binding.pg_batch_count_motifs(h, 4, None, n_graphs=b.n_graphs)
        dt = (time.perf_counter() - t) / reps
        emb = int(counts.sum())
        out["batched_graphs_per_s"] = b.n_graphs / dt
        out["batched_ms"] = 1000 * dt
        out["batched_embeddings_per_s"] = emb / dt
        note(f"batched: {1000 * dt:.1f} ms for {b.n_graphs} graphs")
        # plain path: each graph loaded on its own, one pg_count_motifs call per graph
        rng = np.random.default_rng(6)
        sample = np.sort(rng.choice(b.n_graphs, args.plain_sample, replace=False))
        graphs = [binding.Graph.from_csr(b.graph(int(i))) for i in sample]
        for G in graphs:
            G.motifs(4)
        torch.cuda.synchronize()
        t = time.perf_counter()
        plain = np.stack([G.motifs(4) for G in graphs])
        pdt = time.perf_counter() - t
        for G in graphs:
            G.close()
        note(f"plain: {pdt:.2f} s for {sample.shape[0]} graphs")
        assert np.array_equal(plain, counts[sample]), "plain and batched counts differ"
        # plain path with the same kernel: one pg_batch_count_motifs launch per graph
        binding.pg_batch_count_motifs(h, 4, sample[:8])
        torch.cuda.synchronize()
        t = time.perf_counter()
        same = np.concatenate([binding.pg_batch_count_motifs(h, 4, sample[i:i + 1]) for i in range(sample.shape[0])])
        sdt = time.perf_counter() - t
        note(f"plain, same kernel: {sdt:.2f} s for {sample.shape[0]} graphs")
        assert np.array_equal(same, counts[sample]), "per-graph launches and the batched run differ"
        # the sample's share of the batch's work, to compare like with like
        work = binding.pg_batch_work_estimate(h, b.n_graphs)
        frac = float(work[sample].sum() / work.sum())
        out["plain_sample_graphs"] = int(sample.shape[0])
        out["plain_graphs_per_s"] = sample.shape[0] / pdt
        out["plain_seconds_for_sample"] = pdt
        out["plain_sample_work_fraction"] = frac
        out["batched_over_plain_graphs_per_s"] = out["batched_graphs_per_s"] / out["plain_graphs_per_s"]
        out["plain_same_kernel_graphs_per_s"] = sample.shape[0] / sdt
        out["plain_same_kernel_seconds_for_sample"] = sdt
        out["batched_over_plain_same_kernel"] = out["batched_graphs_per_s"] / out["plain_same_kernel_graphs_per_s"]
        # serving: Poisson arrivals at fractions of the batched capacity
        fp = serve.graph_footprints(b.voff, b.row_ptr)
        srv = serve.Server(h, fp, n_slots=args.serve_slots, max_batch=args.serve_batch, budget_bytes=8 << 30)
        loads = []
        try:
            cap = out["batched_graphs_per_s"]
            for rho in (0.5, 0.8, 0.95):
                ids = rng.integers(0, b.n_graphs, args.serve_requests)
                arr = serve.poisson_arrivals(args.serve_requests, rho * cap, seed=int(rho * 100))
                st = srv.run(ids, arr)
                note(f"served load {rho}: p50 {st.p50_ms:.2f} ms p99 {st.p99_ms:.2f} ms")
                assert np.array_equal(st.results, counts[ids]), "served counts differ from the batched run"
                loads.append({"offered_load": rho, "offered_rate": rho * cap, "requests": st.n_requests,
                              "throughput": st.throughput, "served_over_offered": st.throughput / (rho * cap),
                              "p50_ms": st.p50_ms, "p99_ms": st.p99_ms, "mean_batch": st.mean_batch,
                              "seconds": st.elapsed_s})
        finally:
            srv.close()
        out["serving"] = loads
    finally:
        binding.pg_batch_free(h)
    return out


# the sources that define each workload's kernels (its pipeline file plus the
# shared device helpers and runtime), for keying stored counter readings
KERNEL_FILES = {
    "clique4": ["pg_clique.hip"], "clique5": ["pg_clique.hip"], "tc": ["pg_clique.hip"],
    "motif4": ["pg_motif.hip"], "motif3": ["pg_motif.hip"], "fsm": ["pg_fsm.hip"],
}
COMMON_FILES = ["pg_device.h", "pg_internal.h", "pg_runtime.hip"]


def kernel_source_sha(workload: str = "clique4") -> str:
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1911_06969_amd", "csrc")
    for f in KERNEL_FILES.get(workload, []) + COMMON_FILES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
