#!/usr/bin/env python3
"""Benchmark: end-to-end BCC throughput of the HIP path on one MI355X.

One step = one full solve (First-CC, Rooting, Tagging, Last-CC, heads,
articulation points and canonical edge labels) of a graph already resident
in HBM.  The default workload is the 2^25-vertex R-MAT power-law graph
(edge factor 16, a,b,c = 0.57,0.19,0.19, symmetrised, merged, loops dropped,
ids permuted, int64 offsets).  Throughput is reported in the paper's edge
convention: its Table 1 counts m as directed arcs (both copies of every
undirected edge), so value = arcs / second; undirected edges/s is given too.

Prints ONE JSON line on stdout; a per-kernel table goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload_graph(name):
    from paper_2301_01356_amd import gen

    if name == "rmat":
        return gen.rmat(), {"workload": "rmat25", "n": 1 << 25, "edge_factor": 16, "abc": [0.57, 0.19, 0.19],
                            "offsets": "int64"}
    if name == "grid":
        return gen.grid(), {"workload": "grid4096_p0.7_path4M", "offsets": "int32"}
    if name == "plain":
        return gen.plain(), {"workload": "plain_2^17+pendants+cycles", "offsets": "int32"}
    raise SystemExit(f"unknown workload {name}")


# Algorithmic bytes per launch: each array touched the minimal number of
# times the kernel's definition needs, 4 bytes per gathered word (no cache
# lines).  Offsets are read as int32 inside the solve (int64 input offsets are
# narrowed once).  A = arcs, n = vertices, deg = row lengths, flags = the
# solve's flags (for the tag sample count).
def alg_bytes(kernel, n, A, deg=None, flags=0):
    models = {
        # offsets + adjacency + first[y] per arc + (first, last) of the row vertex
        # + w1/w2 read-modify-write per row + one descendant bit per arc
        "k_tag_sweep": 4 * (n + 1) + 8 * A + 24 * n + A // 8,
        # offsets + adjacency + label write per arc + the 16-byte record of the
        # row vertex (the few exact rows' gathers are left out: a lower bound)
        "k_bcc_label": 4 * (n + 1) + 8 * A + 16 * n,
        # one-pass final labels (sorted rows): the same stream and records
        "k_bcc_final": 4 * (n + 1) + 8 * A + 16 * n,
        # row-wise label fill (sorted loop-free rows): offsets + label write per
        # arc + (label, exact flag) of every row; exact rows' gathers left out
        "k_bcc_rows": 4 * (n + 1) + 4 * A + 8 * n,
        # label read + label write per arc (canonical-label lookups hit the few hot labels)
        "k_bcc_remap4": 8 * A,
    }
    if deg is not None:
        import numpy as np

        from paper_2301_01356_amd import _native as N

        codes = {c: k for k, c in N.TAG_SAMPLE_CODES.items()}
        ks = codes[(flags >> N.TUNE_TAG_SAMPLES_SHIFT) & 0x3]
        live = int((deg > 0).sum())
        # sampled tags: per vertex its one-vertex-tree rank, first[x], offsets,
        # the cleared difference-array slot and the (min, max, vertex) record
        # written by preorder slot; per sampled arc the target and its first[]
        models["k_tag_sample"] = 28 * n + 8 * int(np.minimum(deg, ks).sum())
        # one union-find sampling round: offsets per vertex; per vertex with
        # arcs the sampled target, both sets' parents and the hooking write
        # (finds longer than one hop left out: a lower bound)
        models["k_cc_sample"] = 4 * (n + 1) + 16 * live
    return models.get(kernel)


# Random word accesses per launch that each land on a cache line of their
# own (a lower bound: accesses that happen to share a line, and union-find
# finds longer than one hop, are left out).  Against the measured random-gather
# rate of the GPU these give a kernel's fraction of its line-rate ceiling.
def random_accesses(kernel, n, A, deg=None, flags=0):
    if deg is None:
        return None
    import numpy as np

    from paper_2301_01356_amd import _native as N

    live = int((deg > 0).sum())
    if kernel == "k_tag_sample":
        codes = {c: k for k, c in N.TAG_SAMPLE_CODES.items()}
        ks = codes[(flags >> N.TUNE_TAG_SAMPLES_SHIFT) & 0x3]
        # first[] of every sampled neighbour, and the record written by
        # preorder slot for every vertex with arcs
        return int(np.minimum(deg, ks).sum()) + live
    if kernel == "k_cc_sample":
        # per vertex with arcs: the sampled adjacency word, the parent of the
        # sampled neighbour and the root word that the hook tests and swaps
        return 3 * live
    return None


# HBM traffic of the slowest kernels from two rocprofv3 --pmc runs (FETCH_SIZE,
# WRITE_SIZE; KiB per dispatch) on R-MAT scale 25, and the factors a 1 GiB
# device copy gives the same counters (known bytes / counter).  Valid only for
# the kernel sources and the flags they were taken with; otherwise traffic = null.
COUNTERS = {
    "src_sha": "4bba8af2921599d8",
    "workload": "rmat25",
    "flags": 0x2B32506,
    "copy_factor": {"fetch": 2.0, "write": 1.0},
    "k_bcc_rows": {"fetch_kib": 378484.7, "write_kib": 4090690.0},
    "k_tag_sample": {"fetch_kib": 2381041.1, "write_kib": 1445290.3},
    "k_cc_sample": {"fetch_kib": 2296379.6, "write_kib": 636608.3},
    "k_lr_walk": {"fetch_kib": 1410318.8, "write_kib": 1064381.6},
    "k_rmq_query": {"fetch_kib": 871129.3, "write_kib": 67782.6},
    "k_tree_link": {"fetch_kib": 578806.1, "write_kib": 830754.0},
    "k_mirror_find": {"fetch_kib": 2068277.0, "write_kib": 312027.7},
    "k_lcc_tree": {"fetch_kib": 862361.0, "write_kib": 297084.8},
}


def kernel_src_sha():
    """Hash of the kernel sources without comments and blank space, so that a
    comment edit does not void counters taken on the same code."""
    import hashlib
    import re

    d = os.path.join(ROOT, "paper_2301_01356_amd", "csrc")
    h = hashlib.sha256()
    for f in ("fastbcc.hip", "prims.hpp"):
        with open(os.path.join(d, f), encoding="utf-8") as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def cpu_baseline(sample_scale, g=None, gpu=None):
    """The oracle (Hopcroft-Tarjan, one host thread) on the workload itself
    (``g``, the benchmarked input) or, with a smaller ``sample_scale``, on a
    bounded sample of the same recipe (R-MAT at that scale).  When ``gpu``
    holds the benchmarked solve's (labels, AP flags, #BCC) of ``g``, they must
    equal the oracle's bit for bit."""
    import numpy as np

    import oracle
    from paper_2301_01356_amd import gen

    whole = g is not None
    if not whole:
        g = gen.rmat(scale=sample_scale)
    t0 = time.perf_counter()
    lab, ap, nb, tp, th = oracle.ht_bcc(g.offsets, g.adj)
    wall = time.perf_counter() - t0
    what = (f"the benchmarked R-MAT scale {sample_scale} input itself" if whole else
            f"R-MAT scale {sample_scale} (n=2^{sample_scale}, edge factor 16, same recipe and seed)")
    out = {
        "value": g.num_arcs / wall,
        "unit": "edges/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{what}, {g.num_arcs} arcs, {nb} BCCs; prep {tp:.2f}s + DFS {th:.2f}s",
        "prep_s": round(tp, 3),
        "dfs_s": round(th, 3),
        "seconds": wall,
    }
    if gpu is not None:
        glab, gap, gnb = gpu
        out["gpu_equals_oracle"] = bool(gnb == nb and np.array_equal(gap, ap) and np.array_equal(glab, lab))
    return out


def space_report(workspace_of):
    """Space of the Tarjan-Vishkin explicit skeleton (the second CPU solver,
    paper: the Tarjan-Vishkin appendix and its space comparison) against the
    workspace this library needs, on bounded samples of the workload
    families: the skeleton as a CSR with one vertex per edge of the input
    (4 bytes per offset, 8 per skeleton edge, both directions).  Per-arc
    figures carry the R-MAT sample to the benchmarked size."""
    from oracle.tv_bcc import tv_bcc
    from paper_2301_01356_amd import gen

    rows = []
    for name, g in (("plain", gen.plain()), ("rmat16", gen.rmat(scale=16)),
                    ("grid 256x256 p0.7 + path", gen.grid(seed=12, rows=256, cols=256, path_len=1 << 14)),
                    ("knn10 2^16", gen.family("knn", 1 << 16, 10, seed=6))):
        _, _, _, sz = tv_bcc(g.offsets, g.adj, return_skeleton_size=True)
        skel = 4 * (sz["skeleton_vertices"] + 1) + 8 * sz["skeleton_edges"]
        ws = workspace_of(g.n, g.num_arcs)
        rows.append({"graph": name, "vertices": g.n, "arcs": g.num_arcs, "skeleton_vertices": sz["skeleton_vertices"],
                     "skeleton_edges": sz["skeleton_edges"], "skeleton_bytes": skel, "workspace_bytes": ws,
                     "skeleton_over_workspace": round(skel / ws, 3)})
    return rows


def gather_calibration(table_mib=256, count_log2=28):
    """Random-gather ceiling of this GPU: ``2^count_log2`` int32 reads at
    uniform random positions of a ``table_mib`` MiB table (one per lane, no
    reuse to speak of), timed with events.  Every such read that misses the
    caches moves a whole line, so this rate, not bytes/s, bounds the kernels
    whose work is one random word per item."""
    import torch

    dev = torch.device("cuda:0")
    n_tab = (table_mib << 20) // 4
    cnt = 1 << count_log2
    gen_ = torch.Generator(device=dev)
    gen_.manual_seed(7)
    tab = torch.arange(n_tab, dtype=torch.int32, device=dev)
    idx = torch.randint(0, n_tab, (cnt,), dtype=torch.int32, device=dev, generator=gen_)
    out = torch.empty(cnt, dtype=torch.int32, device=dev)
    for _ in range(2):
        torch.index_select(tab, 0, idx, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record()
    for _ in range(reps):
        torch.index_select(tab, 0, idx, out=out)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ok = bool(torch.equal(out, idx))
    del tab, idx, out
    torch.cuda.empty_cache()
    return {"table_bytes": n_tab * 4, "gathers": cnt, "ms": round(ms, 4), "gathers_per_s": cnt / (ms * 1e-3),
            "stream_bytes_per_s": 8 * cnt / (ms * 1e-3), "result_ok": ok}


# Every generated input has ascending rows and no self-loops; the solve is
# told so (the edge-label read-out then finds reverse arcs by binary search
# and writes labels without re-reading the adjacency).
def _input_flags():
    from paper_2301_01356_amd import _native as N

    return N.FLAG_SORTED_ROWS | N.FLAG_NO_SELF_LOOPS


INPUT_FLAGS = _input_flags()


def tuned_flags(tuner_key, run_once):
    """Autotune the solve's speed-only knobs on this input (outside any timed region)."""
    from paper_2301_01356_amd.tune import Tuner

    t = Tuner(cache_path=None)
    return t.tune(tuner_key, run_once), t.cache[tuner_key]


# Graphs of at most this many vertices go to the fused small-graph kernels
# (packed into runs of at most SMALL_PACK vertices) in the batch leg.
SMALL_SPLIT = 3072
SMALL_PACK = 3072


def bench_tiny_batch(args, dev):
    """Many tiny graphs (16384, n log-uniform in [16, 1024], the batch's
    families): the fused kernels over packs of up to SMALL_PACK vertices
    against the general launch sequence over the same union, both on
    device-resident inputs, results compared on every output."""
    import numpy as np
    import torch

    from paper_2301_01356_amd import _native as N
    from paper_2301_01356_amd import alloc_workspace, gen, solve_batched, solve_small
    from paper_2301_01356_amd.api import greedy_packs

    u = gen.batch(seed=9, count=16384, nmin=16, nmax=1024)
    G = len(u.vbegin) - 1
    vb = torch.from_numpy(u.vbegin).to(dev)
    off = torch.from_numpy(u.offsets32()).to(dev)
    adj = torch.from_numpy(u.adj).to(dev)
    pk = torch.tensor(greedy_packs(np.diff(u.vbegin), SMALL_PACK), dtype=torch.int32, device=dev)
    ws = alloc_workspace(u.n, u.num_arcs, G, dev)

    def timed(fn, steps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / steps

    steps = max(1, args.steps)
    # the general sequence with the defaults and with the per-graph union-find passes: the faster
    general = {fl: timed(lambda: solve_batched(vb, off, adj, workspace=ws, flags=fl), steps)
               for fl in (INPUT_FLAGS, INPUT_FLAGS | N.TUNE_GRAPH_CC)}
    general_flags = min(general, key=general.get)
    ms_general = general[general_flags]
    ms_fused = timed(lambda: solve_small(vb, off, adj, packs=pk, flags=INPUT_FLAGS), steps)
    r1 = solve_small(vb, off, adj, packs=pk, flags=INPUT_FLAGS)
    r2 = solve_batched(vb, off, adj, workspace=ws, flags=general_flags)
    torch.cuda.synchronize()
    same = bool(torch.equal(r1.edge_label, r2.edge_label) and torch.equal(r1.is_ap, r2.is_ap)
                and torch.equal(r1.num_bcc, r2.num_bcc))
    log(f"[bench] tiny graphs ({G}, {u.n} vertices, {u.num_arcs} arcs): general sequence {ms_general:.3f} ms "
        f"(flags {general_flags:#x}; " + ", ".join(f"{k:#x}: {v:.3f} ms" for k, v in general.items()) + "), "
        f"fused kernels over {pk.numel() - 1} packs {ms_fused:.3f} ms, equal={same}")
    del ws, r1, r2
    torch.cuda.empty_cache()
    return {"graphs": G, "vertices": u.n, "arcs": u.num_arcs, "packs": pk.numel() - 1,
            "general_sequence_ms": ms_general, "general_sequence_flags": general_flags, "fused_ms": ms_fused,
            "speedup": ms_general / ms_fused,
            "fused_equals_general": same}


def bench_batch(args):
    """Batched pattern: 4096 graphs (mixed families, n log-uniform in
    [64, 2^16]) against the plain per-graph solve of the same graphs, each
    launched separately.  The batched path splits the batch: graphs of at
    most SMALL_SPLIT vertices go, packed, to the fused one-workgroup-per-pack
    kernels, the rest to the general launch sequence; each part is one
    captured HIP graph on its own stream, so the two overlap.  The general
    sequence over the whole batch is timed beside it."""
    import numpy as np
    import torch

    from paper_2301_01356_amd import gen, solve
    from paper_2301_01356_amd.batch import BatchedSolver, SplitBatchedSolver
    from paper_2301_01356_amd.tune import cache_key, gpu_arch, skew_class

    t0 = time.perf_counter()
    u = gen.batch()
    G = len(u.vbegin) - 1
    graphs = []
    for i in range(G):
        v0, v1 = int(u.vbegin[i]), int(u.vbegin[i + 1])
        a0, a1 = int(u.offsets[v0]), int(u.offsets[v1])
        graphs.append(gen.Csr(v1 - v0, u.offsets[v0 : v1 + 1] - a0, u.adj[a0:a1] - v0))
    log(f"[bench] batch: {G} graphs, n={u.n}, arcs={u.num_arcs}, generated in {time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    cap_v, cap_a = u.n + 1, u.num_arcs
    solver = BatchedSolver(cap_v, cap_a, G, device=dev, use_graph=False)
    solver.stage(graphs)

    def run_once(flags):
        solver.flags = flags | INPUT_FLAGS
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(solver.stream)
        solver._launch()
        e1.record(solver.stream)
        e1.synchronize()
        return e0.elapsed_time(e1)

    solver.launch()  # inputs resident from here on
    solver.done.synchronize()
    key = cache_key(gpu_arch(), u.n, u.num_arcs, G, skew_class(np.diff(u.offsets)))
    flags, cfg = tuned_flags(key, run_once) if not args.flags else (args.flags, {})
    solver.flags = flags | INPUT_FLAGS
    solver.use_graph = True
    solver.graph = None
    solver._ensure_graph()
    s = solver.stream
    with torch.cuda.stream(s):  # a graph replays on the current stream
        for _ in range(args.warmup):
            solver.graph.replay()
        s.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(args.steps):
            solver.graph.replay()
        e1.record(s)
    e1.synchronize()
    ms_general = e0.elapsed_time(e1) / args.steps
    log(f"[bench] batched, general sequence only (graph replay): {ms_general:.3f} ms per batch of {G}")
    # the split path: fused kernels for the small graphs beside the general
    # sequence for the rest, two streams
    small_caps, big_caps = SplitBatchedSolver.capacities(graphs, SMALL_SPLIT)
    split = SplitBatchedSolver(small_caps, big_caps, small_max=SMALL_SPLIT, pack_vertices=SMALL_PACK,
                               device=dev, flags=flags | INPUT_FLAGS)
    split.stage(graphs)
    split.launch()
    split.synchronize()
    n_small = sum(1 for g in graphs if g.n <= SMALL_SPLIT)

    def time_parts(parts, steps):
        cur = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ends = [torch.cuda.Event() for _ in parts]
        e0.record(cur)
        for p in parts:
            p.stream.wait_event(e0)
        for _ in range(steps):
            for p in parts:
                with torch.cuda.stream(p.stream):
                    p.graph.replay()
        for p, e in zip(parts, ends):
            e.record(p.stream)
            cur.wait_event(e)
        e1.record(cur)
        e1.synchronize()
        return e0.elapsed_time(e1) / steps

    split.replay()  # captures both graphs on first use
    split.synchronize()
    time_parts([split.small, split.big], max(1, args.warmup))
    ms_batch = time_parts([split.small, split.big], args.steps)
    ms_small = time_parts([split.small], args.steps)
    ms_big = time_parts([split.big], args.steps)
    log(f"[bench] batched, split (graph replays on two streams): {ms_batch:.3f} ms per batch of {G} "
        f"({n_small} graphs of <= {SMALL_SPLIT} vertices on the fused kernels: {ms_small:.3f} ms alone; "
        f"the other {G - n_small} on the general sequence: {ms_big:.3f} ms alone)")
    from paper_2301_01356_amd import _native as N
    from paper_2301_01356_amd import solve_traced

    tr = N.Trace(max_launches=512)
    solve_traced(solver.d_off, solver.d_adj, tr, vbegin=solver.d_vbegin, out=solver.out, workspace=solver.ws,
                 flags=solver.flags, stream=s)
    tr.collect()
    for name, (t, cnt) in sorted(tr.totals().items(), key=lambda kv: -kv[1][0])[:12]:
        log(f"  {t:9.3f} ms  {cnt:3d} launches  {name}")
    tr.close()

    if getattr(args, "batch_only", False):  # the batched solve alone (for profiling it)
        return {"metric": "batched graphs/s (1 GPU)", "value": G / (ms_batch * 1e-3), "unit": "graphs/s",
                "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_batch,
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
                "data": "synthetic", "config": {"workload": "batch4096_mixed_64..65536", "graphs": G,
                                                "vertices": u.n, "arcs": u.num_arcs, "hip_graph": True,
                                                "tuned": cfg},
                "roofline": None, "cpu_baseline": None}
    # per-graph plain solves (device-resident inputs, one launch sequence each),
    # with the batch's flags and with the defaults: the faster is the baseline
    dgs = [(torch.from_numpy(g.offsets32()).to(dev), torch.from_numpy(g.adj).to(dev)) for g in graphs]
    from paper_2301_01356_amd import alloc_workspace
    from paper_2301_01356_amd.api import BccResult

    maxn = max(g.n for g in graphs)
    maxa = max(g.num_arcs for g in graphs)
    ws = alloc_workspace(maxn, maxa, 1, dev)
    outs = [BccResult(torch.empty(g.num_arcs, dtype=torch.int32, device=dev),
                      torch.empty(g.n, dtype=torch.uint8, device=dev),
                      torch.empty(1, dtype=torch.int64, device=dev)) for g in graphs]
    per_flags = {}
    for pf in (solver.flags, INPUT_FLAGS):
        torch.cuda.synchronize()
        for (o, a), out in zip(dgs[:64], outs[:64]):
            solve(o, a, out=out, workspace=ws, flags=pf)
        torch.cuda.synchronize()
        per = []
        for rep in range(max(1, min(3, args.steps))):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for (o, a), out in zip(dgs, outs):
                solve(o, a, out=out, workspace=ws, flags=pf)
            e1.record()
            e1.synchronize()
            per.append(e0.elapsed_time(e1))
        per_flags[pf] = float(np.median(per))
    per_graph_flags = min(per_flags, key=per_flags.get)
    ms_per_graph_total = per_flags[per_graph_flags]
    log(f"[bench] per-graph plain solves: {ms_per_graph_total:.1f} ms for {G} graphs (flags {per_graph_flags:#x}; "
        + ", ".join(f"{k:#x}: {v:.1f} ms" for k, v in per_flags.items()) + ")")
    tiny = bench_tiny_batch(args, dev)
    # results agree (batched == per-graph) on every graph, for the split
    # path and the general sequence alone
    split.launch()
    br = split.results()
    same = all(np.array_equal(b.edge_label, out.edge_label.cpu().numpy()) and b.num_bcc == int(out.num_bcc.item())
               for b, out in zip(br, outs))
    solver.launch()
    br = solver.results()
    same = same and all(np.array_equal(b.edge_label, out.edge_label.cpu().numpy())
                        and b.num_bcc == int(out.num_bcc.item()) for b, out in zip(br, outs))
    return {
        "metric": "batched vs per-graph speedup (1 GPU)",
        "value": ms_per_graph_total / ms_batch,
        "unit": "x",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_batch,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "batch4096_mixed_64..65536", "graphs": G, "vertices": u.n, "arcs": u.num_arcs,
                   "graphs_per_s": G / (ms_batch * 1e-3), "edges_per_s": u.num_arcs / (ms_batch * 1e-3),
                   "per_graph_total_ms": ms_per_graph_total, "per_graph_flags": per_graph_flags,
                   "hip_graph": True, "tuned": cfg,
                   "general_sequence_only_ms": ms_general,
                   "split": {"small_max_vertices": SMALL_SPLIT, "pack_vertices": SMALL_PACK,
                             "small_graphs": n_small, "small_part_alone_ms": ms_small,
                             "big_part_alone_ms": ms_big},
                   "batched_equals_per_graph": bool(same),
                   "tiny_graphs": tiny},
        "roofline": None,
        "cpu_baseline": None,
    }


def bench_knn_sweep(args):
    """k-NN k-sweep (the shape of the paper's GL2..GL20 rows): 2^22 uniform
    points in the unit square, k in {2, 5, 10, 15, 20}; per k the tuned solve
    time and edges/s (diameter shrinks and edges grow with k)."""
    import numpy as np
    import torch

    from paper_2301_01356_amd import alloc_workspace, gen, solve
    from paper_2301_01356_amd.api import BccResult
    from paper_2301_01356_amd.tune import cache_key, gpu_arch, skew_class

    rows = []
    dev = torch.device("cuda:0")
    for k in (2, 5, 10, 15, 20):
        t0 = time.perf_counter()
        g = gen.config(f"knn{k}")
        off = torch.from_numpy(g.offsets32()).to(dev)
        adj = torch.from_numpy(g.adj).to(dev)
        ws = alloc_workspace(g.n, g.num_arcs, 1, dev)
        out = BccResult(torch.empty(g.num_arcs, dtype=torch.int32, device=dev),
                        torch.empty(g.n, dtype=torch.uint8, device=dev), torch.empty(1, dtype=torch.int64, device=dev))
        st = torch.cuda.current_stream()

        def run_once(f):
            a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a0.record(st)
            solve(off, adj, out=out, workspace=ws, flags=f | INPUT_FLAGS, stream=st)
            a1.record(st)
            a1.synchronize()
            return a0.elapsed_time(a1)

        key = cache_key(gpu_arch(), g.n, g.num_arcs, 1, skew_class(np.diff(g.offsets)))
        flags, cfg = tuned_flags(key, run_once)
        times = [run_once(flags) for _ in range(max(3, args.steps))]
        ms = float(np.median(times))
        rows.append({"k": k, "vertices": g.n, "arcs": g.num_arcs, "ms": ms, "edges_per_s": g.num_arcs / (ms * 1e-3),
                     "num_bcc": int(out.num_bcc.item()), "tuned": cfg})
        log(f"[bench] knn k={k}: {g.num_arcs} arcs, {ms:.3f} ms, {g.num_arcs / ms / 1e6:.2f} G edges/s, "
            f"#BCC={rows[-1]['num_bcc']} (gen {time.perf_counter() - t0:.1f}s)")
        del off, adj, ws, out
        torch.cuda.empty_cache()
    return {
        "metric": "BCC edges/s end-to-end (1 GPU), k-NN k-sweep",
        "value": rows[-1]["edges_per_s"],
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 1,
        "ms_per_step": rows[-1]["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "knn2d_2^22_k2..20", "rows": rows},
        "roofline": None,
        "cpu_baseline": None,
    }


# Serving arrival rate, frozen: 0.7 x the served capacity measured once on
# MI355X (952 graphs/s: 1,500 requests of this pool queued at t = 0, 3 slots,
# the serving flags; the capacity runs of `bench.py --workload serve`).
SERVE_QPS = 665.0


# Table 1 of the paper for its circular grids with p = 0.6 (context: the
# statistics a percolated torus of this shape and size has, whoever solves it)
PAPER_TORI = {"sqr_torus": {"shape": "10^4 x 10^4", "bcc_per_n": 0.2384, "largest_bcc_pct": 70.65},
              "rec_torus": {"shape": "10^3 x 10^5", "bcc_per_n": 0.2383, "largest_bcc_pct": 70.66}}


def bench_tori(args):
    """The paper's SQR' and REC' shapes: percolated tori (p = 0.6) of 10^8
    vertices.  Per torus: the tuned solve's time and edges/s, #BCC / n and the
    largest BCC's share of the vertices (head included), beside Table 1."""
    import numpy as np
    import torch

    from paper_2301_01356_amd import alloc_workspace, gen, read_device_status, solve, vertex_labels
    from paper_2301_01356_amd.api import BccResult
    from paper_2301_01356_amd.tune import cache_key, gpu_arch, skew_class

    rows = []
    dev = torch.device("cuda:0")
    for name in ("sqr_torus", "rec_torus"):
        t0 = time.perf_counter()
        g = gen.config(name)
        off = torch.from_numpy(g.offsets32()).to(dev)
        adj = torch.from_numpy(g.adj).to(dev)
        ws = alloc_workspace(g.n, g.num_arcs, 1, dev)
        out = BccResult(torch.empty(g.num_arcs, dtype=torch.int32, device=dev),
                        torch.empty(g.n, dtype=torch.uint8, device=dev), torch.empty(1, dtype=torch.int64, device=dev))
        st = torch.cuda.current_stream()

        def run_once(f):
            a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a0.record(st)
            solve(off, adj, out=out, workspace=ws, flags=f | INPUT_FLAGS, stream=st)
            a1.record(st)
            a1.synchronize()
            return a0.elapsed_time(a1)

        key = cache_key(gpu_arch(), g.n, g.num_arcs, 1, skew_class(np.diff(g.offsets)))
        flags, cfg = tuned_flags(key, run_once)
        for _ in range(args.warmup):
            run_once(flags)
        times = [run_once(flags) for _ in range(max(3, args.steps))]
        ms = float(np.median(times))
        if read_device_status(ws, st) != 0:
            raise SystemExit(f"[bench] {name}: the solve's device-side checks fired")
        nb = int(out.num_bcc.item())
        home, _ = vertex_labels(ws, g.n, g.num_arcs, stream=st)
        h = home[home >= 0].to(torch.int64)
        largest = int(torch.bincount(h).max().item()) + 1 if h.numel() else 0  # + the BCC's head
        rows.append({"torus": name, "shape": PAPER_TORI[name]["shape"], "vertices": g.n, "arcs": g.num_arcs,
                     "ms": ms, "edges_per_s": g.num_arcs / (ms * 1e-3), "num_bcc": nb,
                     "bcc_per_n": round(nb / g.n, 5), "largest_bcc_pct": round(100.0 * largest / g.n, 3),
                     "paper": PAPER_TORI[name], "flags": flags | INPUT_FLAGS, "tuned": cfg})
        log(f"[bench] {name}: {g.num_arcs} arcs, {ms:.3f} ms, {g.num_arcs / ms / 1e6:.2f} G edges/s, "
            f"#BCC/n {nb / g.n:.4f} (paper {PAPER_TORI[name]['bcc_per_n']}), largest BCC "
            f"{100.0 * largest / g.n:.2f}% (paper {PAPER_TORI[name]['largest_bcc_pct']}%), "
            f"gen {time.perf_counter() - t0:.1f}s")
        del off, adj, ws, out, home, h
        torch.cuda.empty_cache()
    return {
        "metric": "BCC edges/s end-to-end (1 GPU), paper-shaped tori",
        "value": rows[0]["edges_per_s"],
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rows[0]["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "tori_p0.6_10^8", "rows": rows},
        "roofline": None,
        "cpu_baseline": None,
    }


def pinned_link_rates(dev, mib=64, reps=10):
    """Pinned host <-> device copy rates of this machine (torch copies on two
    streams): host to device alone, device to host alone, and both at once
    (total).  Requests of a server cross this link twice."""
    import torch

    count = mib << 18
    h1 = torch.empty(count, dtype=torch.int32, pin_memory=True)
    h2 = torch.empty(count, dtype=torch.int32, pin_memory=True)
    d1 = torch.empty(count, dtype=torch.int32, device=dev)
    d2 = torch.empty(count, dtype=torch.int32, device=dev)
    s1, s2 = torch.cuda.Stream(device=dev), torch.cuda.Stream(device=dev)

    def h2d():
        with torch.cuda.stream(s1):
            d1.copy_(h1, non_blocking=True)

    def d2h():
        with torch.cuda.stream(s2):
            h2.copy_(d2, non_blocking=True)

    def rate(fns):
        for f in fns:
            f()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            for f in fns:
                f()
        torch.cuda.synchronize()
        return reps * len(fns) * count * 4 / (time.perf_counter() - t) / 1e9

    out = {"h2d_GBps": rate([h2d]), "d2h_GBps": rate([d2h]), "both_total_GBps": rate([h2d, d2h])}
    del h1, h2, d1, d2
    return out


def bench_serve(args):
    """Serving: Poisson arrivals at a frozen rate of mixed-family requests
    (n log-uniform in [2^10, 2^22], mean degree 4-32), for at least a minute;
    continuous batching over HIP streams, admission by live free HBM; p50/p99
    latency, against serial plain solves of the same request stream."""
    import numpy as np
    import torch

    import oracle
    from paper_2301_01356_amd import gen
    from paper_2301_01356_amd.batch import PinnedGraph
    from paper_2301_01356_amd.serve import (PlainSlot, Request, Server, hip_slots, latency_summary,
                                            poisson_arrivals, serving_flags)

    t0 = time.perf_counter()
    # a pool of distinct request graphs in pinned host memory; each request
    # draws one (seeded), as a stream of independent queries would
    pool_src = [gen.mixed(5, i, 1 << 10, 1 << 22, 4.0, 32.0) for i in range(args.serve_pool)]
    pool = [PinnedGraph(g) for g in pool_src]
    log(f"[bench] serve: pool of {len(pool)} graphs, {sum(g.num_arcs for g in pool)} arcs, "
        f"generated in {time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    maxn = max(g.n for g in pool)
    maxa = max(g.num_arcs for g in pool)
    cap_v = max(1 << 23, 2 * maxn + 2)
    cap_a = max(1 << 27, 2 * maxa)
    flags = serving_flags()
    slots = hip_slots(args.slots, cap_v, cap_a, 64, flags=flags, digests=True)
    serial_slot = PlainSlot(maxn + 1, maxa, flags=flags, digests=True)
    for sl in slots + [serial_slot]:  # warm every slot once
        sl.launch(pool[:1])
        sl.results()
    free0, total_b = torch.cuda.mem_get_info()
    budget = int(free0 * 0.6)
    def live_free():
        return torch.cuda.mem_get_info()[0]

    def stream_of(count, arrivals, seed):
        pick = np.random.default_rng(seed).integers(len(pool), size=count)
        return [Request(i, pool[pick[i]], float(arrivals[i])) for i in range(count)], pick

    keep_every = 97

    def run(reqs, srv_slots, max_batch=None):
        srv = Server(srv_slots, budget, max_batch_graphs=max_batch, free_hbm=live_free,
                     keep=lambda r: r.rid % keep_every == 0)
        t = time.perf_counter()
        comps = srv.run(reqs)
        return comps, srv.stats, time.perf_counter() - t

    qps = args.qps or SERVE_QPS
    # capacities: the same requests all queued at t = 0, served (continuous
    # batching over the slots) and serial (one plain solve at a time)
    n_cap = args.capacity_requests
    # warm-up: the first batches of each kind allocate the temporaries that the
    # caching allocator then keeps
    warm, _ = stream_of(200, np.zeros(200), 49)
    run(warm, slots)
    run(warm[:50], [serial_slot], max_batch=1)
    reqs, _ = stream_of(n_cap, np.zeros(n_cap), 50)

    def set_digests(on):  # the verification fingerprints are GPU work that serving does not do
        for sl in slots:
            sl.solver.digests = on
        serial_slot.digests = on

    set_digests(False)
    comps_t, st, wall = run(reqs, slots)
    cap = n_cap / wall
    log(f"[bench] served capacity {cap:.1f} graphs/s ({n_cap} requests queued at t=0, {st['batches']} batches)")
    comps_c1t, _, wall_c1 = run(reqs, [serial_slot], max_batch=1)
    cap_serial = n_cap / wall_c1
    log(f"[bench] serial capacity {cap_serial:.1f} graphs/s")
    link = pinned_link_rates(dev)
    # bytes a request moves: its CSR in (row starts and arcs), its labels,
    # AP flags and count out
    in_bytes = float(np.mean([4 * r.graph.num_arcs + 4 * (r.graph.n + 1) for r in reqs]))
    out_bytes = float(np.mean([4 * r.graph.num_arcs + r.graph.n + 20 for r in reqs]))
    req_bytes = in_bytes + out_bytes
    link_bound = min(link["h2d_GBps"] * 1e9 / in_bytes, link["d2h_GBps"] * 1e9 / out_bytes,
                     link["both_total_GBps"] * 1e9 / req_bytes)
    log(f"[bench] pinned link: H2D {link['h2d_GBps']:.1f} GB/s, D2H {link['d2h_GBps']:.1f} GB/s, both at once "
        f"{link['both_total_GBps']:.1f} GB/s total; {req_bytes / 1e6:.1f} MB per request -> at most "
        f"{link_bound:.0f} graphs/s over the link (served: {100 * cap / link_bound:.0f}% of it)")
    set_digests(True)
    # the same two runs again with fingerprints, untimed, to check them equal
    comps, _, _ = run(reqs, slots)
    comps_c1, _, _ = run(reqs, [serial_slot], max_batch=1)
    same_cap = all(a.ok and b.ok and a.digest == b.digest and a.num_bcc == b.num_bcc
                   for a, b in zip(comps, comps_c1))
    same_cap = same_cap and all(a.ok and b.ok and a.num_bcc == c.num_bcc == b.num_bcc
                                for a, b, c in zip(comps_t, comps_c1t, comps))
    if qps is None:
        qps = 0.7 * cap
    count = max(int(np.ceil(qps * args.serve_seconds)), 1)
    arr = poisson_arrivals(count, qps, 5)
    reqs, pick = stream_of(count, arr, 5)
    log(f"[bench] serve: {count} requests at {qps:.1f} QPS (Poisson) over {arr[-1]:.1f}s")
    comps, st, wall = run(reqs, slots)
    s_mix = latency_summary(comps)
    ok = all(c.ok for c in comps)
    log(f"[bench] served: p50 {s_mix['p50_ms']:.2f} ms p99 {s_mix['p99_ms']:.2f} ms, "
        f"{s_mix['graphs_per_s']:.1f} graphs/s, {st['batches']} batches, wall {wall:.1f}s")
    # serial plain solves of the same stream (its first requests): one at a
    # time, each with only its own copies and a workspace sized for it
    n_ser = min(count, args.serial_requests)
    comps1, st1, wall1 = run(reqs[:n_ser], [serial_slot], max_batch=1)
    s_ser = latency_summary(comps1)
    log(f"[bench] serial ({n_ser} requests): p50 {s_ser['p50_ms']:.2f} ms p99 {s_ser['p99_ms']:.2f} ms, "
        f"{s_ser['graphs_per_s']:.1f} graphs/s")
    same = same_cap and all(a.ok and b.ok and a.digest == b.digest and a.num_bcc == b.num_bcc
                            for a, b in zip(comps[:n_ser], comps1))
    # the kept results against the oracle, one per distinct pool graph
    checked, agree, seen = 0, True, set()
    for c in comps:
        p = int(pick[c.rid])
        if c.edge_label is None or p in seen or len(seen) >= args.serve_oracle_checks:
            continue
        seen.add(p)
        lab, ap, nb, _, _ = oracle.ht_bcc(pool_src[p].offsets, pool_src[p].adj)
        agree = agree and bool(np.array_equal(c.edge_label, lab) and np.array_equal(c.is_ap, ap) and c.num_bcc == nb)
        checked += 1
    log(f"[bench] served == serial on {n_cap} + {n_ser} requests: {same}; {checked} kept results == oracle: {agree}")
    return {
        "metric": "serving p50/p99 latency and graphs/s (1 GPU)",
        "value": s_mix["graphs_per_s"],
        "unit": "graphs/s",
        "n_gpus": 1,
        "steps": count,
        "warmup": args.slots + 1,
        "ms_per_step": 1e3 / s_mix["graphs_per_s"] if s_mix["graphs_per_s"] else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "serve_mixed_2^10..2^22", "requests": count, "pool_graphs": len(pool),
                   "pool_arcs": sum(g.num_arcs for g in pool), "qps": qps,
                   "qps_source": "frozen" if (args.qps or SERVE_QPS) else "0.7 x capacity measured in this run",
                   "arrival_span_s": float(arr[-1]), "flags": flags, "input_contract": "general",
                   "capacity_graphs_per_s": cap, "serial_capacity_graphs_per_s": cap_serial,
                   "pinned_link": link, "bytes_per_request": req_bytes,
                   "link_bound_graphs_per_s": link_bound, "served_fraction_of_link_bound": cap / link_bound,
                   "capacity_requests": n_cap, "served_vs_serial_capacity": cap / cap_serial,
                   "slots": args.slots, "hbm_budget_bytes_initial": budget,
                   "hbm_budget_bytes_min": st["min_budget"], "budget_reads": st["budget_reads"],
                   "served": s_mix, "batches": st["batches"], "max_queue": st["max_queue"],
                   "serial": dict(s_ser, requests=n_ser, wall_s=wall1),
                   "all_ok": ok, "served_equals_serial": bool(same), "oracle_checked": checked,
                   "oracle_agrees": bool(agree)},
        "roofline": None,
        "cpu_baseline": None,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat", choices=["rmat", "grid", "plain", "batch", "serve", "knn_sweep", "tori"])
    ap.add_argument("--slots", type=int, default=3)
    ap.add_argument("--qps", type=float, default=0.0, help="serving arrival rate (default: the frozen rate)")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="serving: seconds of Poisson arrivals")
    ap.add_argument("--serve-pool", type=int, default=64, help="serving: distinct request graphs")
    ap.add_argument("--serial-requests", type=int, default=1000, help="serving: requests of the serial baseline")
    ap.add_argument("--serve-oracle-checks", type=int, default=6)
    ap.add_argument("--capacity-requests", type=int, default=1500, help="serving: requests of the capacity runs")
    ap.add_argument("--cpu-sample-scale", type=int, default=25,
                    help="25: the oracle runs on the benchmarked R-MAT input itself and is compared with the GPU")
    ap.add_argument("--no-gather-calibration", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--flags", type=lambda s: int(s, 0), default=0)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="skip the HIP-graph replay timing")
    ap.add_argument("--batch-only", action="store_true", help="batch workload: the batched solve alone")
    ap.add_argument("--no-systems", action="store_true", help="skip the batched and serving legs")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration under rocprofv3)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library solves a graph on one GPU and has no "
              "multi-GPU path (the design notes describe how the solve would shard).", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration_mib:
        import torch

        nb = args.copy_calibration_mib << 20
        src = torch.ones(nb // 4, dtype=torch.int32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: 3 x {nb} bytes read + {nb} bytes written")
        del src, dst
    if args.workload == "batch":
        print(json.dumps(bench_batch(args)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(bench_serve(args)), flush=True)
        return
    if args.workload == "knn_sweep":
        print(json.dumps(bench_knn_sweep(args)), flush=True)
        return
    if args.workload == "tori":
        print(json.dumps(bench_tori(args)), flush=True)
        return

    import torch

    from paper_2301_01356_amd import _native as N
    from paper_2301_01356_amd import alloc_workspace, solve, solve_traced
    from paper_2301_01356_amd.api import BccResult

    t0 = time.perf_counter()
    g, cfg = workload_graph(args.workload)
    log(f"[bench] generated {cfg['workload']}: n={g.n} arcs={g.num_arcs} in {time.perf_counter() - t0:.1f}s")
    dev = torch.device("cuda:0")
    off64 = cfg["offsets"] == "int64"
    off = torch.from_numpy(g.offsets if off64 else g.offsets32()).to(dev)
    adj = torch.from_numpy(g.adj).to(dev)
    n, A = g.n, g.num_arcs
    deg = (g.offsets[1:] - g.offsets[:-1]).astype("int64")  # row lengths, for the byte models
    ws = alloc_workspace(n, A, 1, dev)
    out = BccResult(
        torch.empty(A, dtype=torch.int32, device=dev),
        torch.empty(n, dtype=torch.uint8, device=dev),
        torch.empty(1, dtype=torch.int64, device=dev),
    )
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    tuned = {}
    if not args.flags and not args.no_tune:
        import numpy as np

        from paper_2301_01356_amd.tune import cache_key, gpu_arch, skew_class

        def run_once(f):
            a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a0.record(stream)
            solve(off, adj, out=out, workspace=ws, flags=f | INPUT_FLAGS, stream=stream)
            a1.record(stream)
            a1.synchronize()
            return a0.elapsed_time(a1)

        key = cache_key(gpu_arch(), n, A, 1, skew_class(np.diff(g.offsets)))
        args.flags, tuned = tuned_flags(key, run_once)
        log(f"[bench] tuned flags {args.flags:#x}: {tuned}")
    args.flags |= INPUT_FLAGS

    for _ in range(args.warmup):
        solve(off, adj, out=out, workspace=ws, flags=args.flags, stream=stream)
    torch.cuda.synchronize()
    log(f"[bench] warmup done ({args.warmup} steps)")

    # timed region: K plain solves bracketed by events on the solve's stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        solve(off, adj, out=out, workspace=ws, flags=args.flags, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    num_bcc = int(out.num_bcc.item())
    log(f"[bench] {args.steps} steps: {ms:.3f} ms/step, {A / ms / 1e6:.2f} G arcs/s, #BCC={num_bcc}")
    from paper_2301_01356_amd import read_device_status

    status = read_device_status(ws, stream)
    if status != 0:
        raise SystemExit(f"[bench] the solve's device-side checks fired (status {status})")

    # what the input promises buy: the same solve under the general input
    # contract (rows in any order, self-loops allowed), and with the device
    # validation pass in front (which synchronises the host once per solve)
    ref_label = out.edge_label.clone()
    contract = {}
    for what, f in (("general_contract", args.flags & ~INPUT_FLAGS), ("validated", args.flags | N.FLAG_VALIDATE)):
        solve(off, adj, out=out, workspace=ws, flags=f, stream=stream)
        torch.cuda.synchronize()
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record(stream)
        for _ in range(args.steps):
            solve(off, adj, out=out, workspace=ws, flags=f, stream=stream)
        c1.record(stream)
        torch.cuda.synchronize()
        same = bool(torch.equal(out.edge_label, ref_label)) and int(out.num_bcc.item()) == num_bcc
        if not same or read_device_status(ws, stream) != 0:
            raise SystemExit(f"[bench] the {what} solve disagrees with the benchmarked one")
        contract[what] = {"flags": f, "ms_per_step": c0.elapsed_time(c1) / args.steps, "same_result": same}
        log(f"[bench] {what}: {contract[what]['ms_per_step']:.3f} ms/step (flags {f:#x})")
    del ref_label

    # the same solve captured once into a HIP graph (the solve enqueues
    # kernels only) and replayed K times: the launch gaps between its kernels
    # go away; the labels must equal the eager ones
    ms_graph = None
    if not args.no_graph:
        ref_label = out.edge_label.clone()
        gs = torch.cuda.Stream()
        gs.wait_stream(stream)
        with torch.cuda.stream(gs):
            hg = torch.cuda.CUDAGraph()
            with torch.cuda.graph(hg, stream=gs):
                solve(off, adj, out=out, workspace=ws, flags=args.flags, stream=gs)
            for _ in range(args.warmup):
                hg.replay()
            out.edge_label.fill_(-7)
            hg.replay()
        gs.synchronize()
        if not torch.equal(out.edge_label, ref_label) or int(out.num_bcc.item()) != num_bcc:
            raise SystemExit("[bench] graph replay disagrees with the eager solve")
        del ref_label
        g0 = torch.cuda.Event(enable_timing=True)
        g1 = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(gs):
            g0.record(gs)
            for _ in range(args.steps):
                hg.replay()
            g1.record(gs)
        gs.synchronize()
        ms_graph = g0.elapsed_time(g1) / args.steps
        log(f"[bench] {args.steps} graph replays: {ms_graph:.3f} ms/step, {A / ms_graph / 1e6:.2f} G arcs/s")
        stream.wait_stream(gs)
        torch.cuda.synchronize()

    # per-kernel durations: the same K steps with an event pair per launch
    tr = N.Trace(max_launches=256 * args.steps + 256)
    for _ in range(args.steps):
        solve_traced(off, adj, tr, out=out, workspace=ws, flags=args.flags, stream=stream)
    tr.collect()
    tot = tr.totals()
    rows = sorted(tot.items(), key=lambda kv: -kv[1][0])
    traced_ms = sum(v[0] for v in tot.values()) / args.steps
    log(f"[bench] traced: kernel time per step {traced_ms:.3f} ms")
    for name, (t, cnt) in rows:
        log(f"  {t / args.steps:9.3f} ms/step  {cnt // args.steps:4d} launches/step  {name}")
    dom_name, (dom_ms, dom_cnt) = rows[0]
    modelled = []
    for name, (t, cnt) in rows:
        b = alg_bytes(name, n, A, deg, args.flags)
        if b is None:
            continue
        avg_ms = t / cnt
        achieved = b / (avg_ms * 1e-3) / 1e9
        traffic = traffic_raw = None
        c = COUNTERS.get(name)
        if (c and cfg["workload"] == COUNTERS["workload"] and kernel_src_sha() == COUNTERS["src_sha"]
                and args.flags == COUNTERS["flags"]):
            f = COUNTERS["copy_factor"]
            traffic = (c["fetch_kib"] * f["fetch"] + c["write_kib"] * f["write"]) * 1024
            traffic_raw = (c["fetch_kib"] + c["write_kib"]) * 1024
        modelled.append({
            "kernel": name,
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "traffic_raw_counters": traffic_raw,
            "traffic_GBps": round(traffic_raw / (avg_ms * 1e-3) / 1e9, 1) if traffic_raw else None,
            "alg_bytes_per_launch": int(b),
            "avg_launch_ms": round(avg_ms, 4),
            "share_of_step": round((t / args.steps) / ms, 3),
        })
    roofline = modelled[0] if modelled else None
    if roofline and roofline["kernel"] != dom_name:
        roofline["note"] = f"slowest kernel {dom_name} has no byte model; reported the slowest modelled one"

    gather = None
    if not args.no_gather_calibration:
        gather = gather_calibration()
        log(f"[bench] random-gather calibration: {gather['gathers_per_s'] / 1e9:.1f} G gathers/s "
            f"from a {gather['table_bytes'] >> 20} MiB table")
        for r in [roofline] + modelled[1:3]:
            lines = r and random_accesses(r["kernel"], n, A, deg, args.flags)
            if lines:
                rate = lines / (r["avg_launch_ms"] * 1e-3)
                r["random_accesses_per_launch"] = int(lines)
                r["line_rate_frac"] = round(rate / gather["gathers_per_s"], 4)

    cpu = None
    if not args.no_cpu_baseline:
        whole = args.workload == "rmat" and args.cpu_sample_scale == 25
        log(f"[bench] CPU oracle on {'the benchmarked input' if whole else f'R-MAT scale {args.cpu_sample_scale}'} ...")
        gpu_res = (out.edge_label.cpu().numpy(), out.is_ap.cpu().numpy(), num_bcc) if whole else None
        cpu = cpu_baseline(args.cpu_sample_scale, g if whole else None, gpu_res)
        del gpu_res
        log(f"[bench] CPU oracle: {cpu['value'] / 1e6:.1f} M arcs/s in {cpu['seconds']:.1f}s"
            + (f", GPU == oracle: {cpu['gpu_equals_oracle']}" if whole else ""))
        del cpu["seconds"]
        t_sp = time.perf_counter()
        cpu["space_report"] = space_report(lambda nn, aa: N.workspace_size(nn, aa, 1))
        r16 = next(r for r in cpu["space_report"] if r["graph"] == "rmat16")
        skel25 = r16["skeleton_bytes"] / r16["arcs"] * A
        cpu["space_report_rmat25_extrapolated"] = {"skeleton_bytes": int(skel25), "workspace_bytes": int(ws.numel()),
                                                   "skeleton_over_workspace": round(skel25 / ws.numel(), 3)}
        log(f"[bench] space report ({time.perf_counter() - t_sp:.1f}s): "
            + ", ".join(f"{r['graph']} {r['skeleton_over_workspace']}x" for r in cpu["space_report"]))
        if whole and not cpu["gpu_equals_oracle"]:
            raise SystemExit("[bench] the benchmarked solve differs from the oracle")

    value = A / (ms * 1e-3)
    line = {
        "metric": "BCC edges/s end-to-end (1 GPU)",
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {**cfg, "arcs": A, "vertices": n, "num_bcc": num_bcc, "flags": args.flags, "tuned": tuned,
                   "edge_convention": "directed arcs (paper Table 1 m)",
                   "undirected_edges_per_s": value / 2, "parallelism": "single GPU",
                   "hip_graph_ms_per_step": ms_graph,
                   "hip_graph_edges_per_s": A / (ms_graph * 1e-3) if ms_graph else None,
                   "general_contract_ms_per_step": contract["general_contract"]["ms_per_step"],
                   "validated_ms_per_step": contract["validated"]["ms_per_step"], "contract": contract},
        "roofline": roofline,
        "rooflines_next": modelled[1:3],
        "gather_calibration": gather,
        "cpu_baseline": cpu,
    }
    if not args.no_systems and args.workload == "rmat":
        del g, off, adj, ws, out
        torch.cuda.empty_cache()
        sys_args = argparse.Namespace(**{**vars(args), "flags": 0})
        b = bench_batch(sys_args)
        line["batched"] = {"speedup_vs_per_graph": b["value"], "ms_per_batch": b["ms_per_step"], **b["config"]}
        torch.cuda.empty_cache()
        sv = bench_serve(sys_args)
        line["serving"] = {"graphs_per_s": sv["value"], **sv["config"]}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
