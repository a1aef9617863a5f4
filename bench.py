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
# lines).  o = offset width, A = arcs, n = vertices.
def alg_bytes(kernel, n, A, o):
    k = kernel.split("<")[0].strip("()")
    models = {
        # offsets + adjacency + first[y] per arc + w1/w2 read-modify-write per row
        "k_tag_sweep": o * (n + 1) + 8 * A + 16 * n,
        # offsets + adjacency + {first, label}[y] per arc + label write per arc + {first, label}[x] per row
        "k_bcc_output": o * (n + 1) + 16 * A + 8 * n,
        # offsets + adjacency + rec[y] (first, last, parent: 12 B) per arc + lab[x] per row
        "k_lcc_sweep": o * (n + 1) + 16 * A + 4 * n,
        # offsets + adjacency + cc[x] per row
        "k_cc_sweep": o * (n + 1) + 4 * A + 4 * n,
        # offsets + adjacency of candidate rows (upper bound: all) + rec/lab gathers
        "k_bcc_minid": o * (n + 1) + 12 * A + n,
    }
    return models.get(k)


def cpu_baseline(sample_scale):
    """The oracle (Hopcroft-Tarjan, one host thread) on a bounded sample of
    the same workload recipe: R-MAT at a smaller scale."""
    import oracle
    from paper_2301_01356_amd import gen

    g = gen.rmat(scale=sample_scale)
    t0 = time.perf_counter()
    _, _, nb, tp, th = oracle.ht_bcc(g.offsets, g.adj)
    wall = time.perf_counter() - t0
    return {
        "value": g.num_arcs / wall,
        "unit": "edges/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"R-MAT scale {sample_scale} (n=2^{sample_scale}, edge factor 16, same recipe and seed), "
        f"{g.num_arcs} arcs, {nb} BCCs; prep {tp:.2f}s + DFS {th:.2f}s",
        "seconds": wall,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat", choices=["rmat", "grid", "plain"])
    ap.add_argument("--cpu-sample-scale", type=int, default=22)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--flags", type=lambda s: int(s, 0), default=0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the design notes describe how the solve would shard).", file=sys.stderr)
        sys.exit(2)

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
    ws = alloc_workspace(n, A, 1, dev)
    out = BccResult(
        torch.empty(A, dtype=torch.int32, device=dev),
        torch.empty(n, dtype=torch.uint8, device=dev),
        torch.empty(1, dtype=torch.int64, device=dev),
    )
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

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

    # per-kernel durations: the same K steps with an event pair per launch
    tr = N.Trace(max_launches=256 * args.steps + 256)
    for _ in range(args.steps):
        solve_traced(off, adj, tr, out=out, workspace=ws, flags=args.flags, stream=stream)
    tr.collect()
    tot = tr.totals()
    rows = sorted(tot.items(), key=lambda kv: -kv[1][0])
    traced_ms = sum(v[0] for v in tot.values()) / args.steps
    log(f"[bench] traced: kernel time per step {traced_ms:.3f} ms")
    for name, (t, cnt) in rows[:25]:
        log(f"  {t / args.steps:9.3f} ms/step  {cnt // args.steps:4d} launches/step  {name}")
    dom_name, (dom_ms, dom_cnt) = rows[0]
    o = 8 if off64 else 4
    roofline = None
    for name, (t, cnt) in rows:
        b = alg_bytes(name, n, A, o)
        if b is None:
            continue
        avg_ms = t / cnt
        achieved = b / (avg_ms * 1e-3) / 1e9
        roofline = {
            "kernel": name,
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "alg_bytes_per_launch": int(b),
            "avg_launch_ms": round(avg_ms, 4),
            "share_of_step": round((t / args.steps) / ms, 3),
        }
        break
    if roofline and roofline["kernel"] != dom_name:
        roofline["note"] = f"slowest kernel {dom_name} has no byte model; reported the slowest modelled one"

    cpu = None
    if not args.no_cpu_baseline:
        log(f"[bench] CPU oracle on R-MAT scale {args.cpu_sample_scale} ...")
        cpu = cpu_baseline(args.cpu_sample_scale)
        log(f"[bench] CPU oracle: {cpu['value'] / 1e6:.1f} M arcs/s in {cpu['seconds']:.1f}s")
        del cpu["seconds"]

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
        "config": {**cfg, "arcs": A, "vertices": n, "num_bcc": num_bcc,
                   "edge_convention": "directed arcs (paper Table 1 m)",
                   "undirected_edges_per_s": value / 2, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
