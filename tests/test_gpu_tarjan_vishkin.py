"""The HIP path against the second, independent CPU solver: Tarjan-Vishkin
with an explicit skeleton (paper: the Tarjan-Vishkin appendix), which shares
neither method nor code with the Hopcroft-Tarjan oracle or the GPU path.
Medium graphs of every workload family, multigraphs with self-loops and
shuffled rows, and the benchmark's input promises; bit-exact labels,
articulation points and BCC counts."""
import sys

import numpy as np
import pytest
import torch

from oracle.tv_bcc import tv_bcc
from paper_2301_01356_amd import _native as N
from paper_2301_01356_amd import alloc_workspace, gen, read_device_status, solve
from paper_2301_01356_amd.tune import shipped_entries

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
PROMISES = N.FLAG_SORTED_ROWS | N.FLAG_NO_SELF_LOOPS


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def hip(g, flags):
    off = torch.from_numpy(g.offsets32()).to(DEV)
    adj = torch.from_numpy(g.adj).to(DEV)
    ws = alloc_workspace(g.n, g.num_arcs, 1, DEV)
    r = solve(off, adj, workspace=ws, flags=flags)
    assert read_device_status(ws) == 0
    return r.edge_label.cpu().numpy(), r.is_ap.cpu().numpy(), int(r.num_bcc.item())


def graphs():
    yield "plain", gen.config("plain")
    yield "grid_small", gen.config("grid_small")
    yield "rmat16", gen.rmat(seed=31, scale=16)
    yield "batch_small_union", gen.config("batch_small")
    yield "knn5_2^16", gen.family("knn", 1 << 16, 5, seed=32)
    yield "lattice_p0.6", gen.family("lattice", 1 << 16, 0.6, seed=33)
    yield "tree_back", gen.family("tree_back", 1 << 16, 0.2, seed=34)


@pytest.mark.parametrize("name,g", list(graphs()), ids=[n for n, _ in graphs()])
def test_hip_equals_tarjan_vishkin(name, g):
    note(f"Tarjan-Vishkin {name} n={g.n} arcs={g.num_arcs}")
    tlab, tap, tnb = tv_bcc(g.offsets, g.adj)
    for flags in (0, shipped_entries()["rmat25"][0] | PROMISES, shipped_entries()["grid"][0] | PROMISES):
        note(f"HIP {name} flags={flags:#x}")
        lab, ap, nb = hip(g, flags)
        assert nb == tnb, f"{name} {flags:#x}: {nb} BCCs, Tarjan-Vishkin {tnb}"
        assert np.array_equal(ap, tap), f"{name} {flags:#x}: articulation points differ"
        bad = np.flatnonzero(lab != tlab)
        assert bad.size == 0, f"{name} {flags:#x}: {bad.size} labels differ"


def test_hip_equals_tarjan_vishkin_multigraphs():
    rng = np.random.default_rng(35)
    for t in range(30):
        n = int(rng.integers(2, 300))
        edges = [(int(rng.integers(0, n)), int(rng.integers(0, n))) for _ in range(int(rng.integers(0, 3 * n)))]
        edges += edges[: int(rng.integers(0, 8))]
        g = gen.multigraph_csr(n, edges)
        adj = g.adj.copy()
        for v in range(n):
            a, b = g.offsets[v], g.offsets[v + 1]
            adj[a:b] = rng.permutation(adj[a:b])
        g = gen.Csr(n, g.offsets, adj)
        note(f"Tarjan-Vishkin multigraph #{t} n={n} arcs={g.num_arcs}")
        tlab, tap, tnb = tv_bcc(g.offsets, g.adj)
        lab, ap, nb = hip(g, 0)
        assert nb == tnb and np.array_equal(ap, tap) and np.array_equal(lab, tlab), f"multigraph {t}"
