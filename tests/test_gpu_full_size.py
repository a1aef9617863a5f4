"""Full-size parity: every benchmark workload at its real size, in the launch
configurations the benchmark times -- the tuned flags shipped in
``tuned_gfx950.json`` together with the input promises every generated graph
keeps (ascending, loop-free rows) -- against the full CPU oracle.  The same
inputs also run under the general input contract (no promises) and with
device-side validation.  After every solve the device status word (the
solve's in-kernel invariant checks) must read 0."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2301_01356_amd import _native as N
from paper_2301_01356_amd import alloc_workspace, gen, read_device_status, solve, solve_batched
from paper_2301_01356_amd.tune import SHIP_WORKLOADS, shipped_entries

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
PROMISES = N.FLAG_SORTED_ROWS | N.FLAG_NO_SELF_LOOPS
SHIPPED = shipped_entries()


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def shipped_flags(name):
    assert name in SHIPPED, f"no shipped tuning entry for the {name} workload"
    return SHIPPED[name][0]


def gpu_solve(g, flags, off64=False):
    off = torch.from_numpy(g.offsets if off64 else g.offsets32()).to(DEV)
    adj = torch.from_numpy(g.adj).to(DEV)
    ws = alloc_workspace(g.n, g.num_arcs, 1, DEV)
    r = solve(off, adj, workspace=ws, flags=flags)
    assert read_device_status(ws) == 0, f"a device-side invariant check fired (flags {flags:#x})"
    got = (r.edge_label.cpu().numpy(), r.is_ap.cpu().numpy(), int(r.num_bcc.item()))
    del off, adj, ws, r
    torch.cuda.empty_cache()
    return got


def assert_same(ref, got, what):
    lab, ap, nb = ref
    glab, gap, gnb = got
    assert gnb == nb, f"{what}: num_bcc {gnb} != {nb}"
    assert np.array_equal(gap, ap), f"{what}: articulation points differ"
    bad = np.flatnonzero(glab != lab)
    assert bad.size == 0, f"{what}: {bad.size} labels differ, first at arc {bad[0]}"


def run_single(name, g, off64, flag_sets):
    outs = []
    for what, flags in flag_sets:
        note(f"{name}: GPU solve ({what}) flags={flags:#x}")
        outs.append((what, flags, gpu_solve(g, flags, off64)))
    note(f"{name}: oracle")
    lab, ap, nb, _, _ = oracle.ht_bcc(g.offsets, g.adj)
    for what, flags, got in outs:
        assert_same((lab, ap, nb), got, f"{name} {what} {flags:#x}")


def test_rmat25_full_size_exact():
    """The headline input: the benchmarked configuration (shipped flags with
    the input promises, int64 offsets), the same flags under the general
    input contract and with validation, the defaults, and other variants."""
    f = shipped_flags("rmat25")
    note("R-MAT scale 25: generate")
    g = gen.rmat()
    run_single("R-MAT scale 25", g, True, [
        ("benchmarked", f | PROMISES),
        ("general contract", f),
        ("validated", f | PROMISES | N.FLAG_VALIDATE),
        ("defaults", 0),
        ("priority union-find, exact tags", N.FLAG_SORTED_ROWS
         | N.tune_flags(ruler_shift=6, sample_rounds=2, tile_shift=4, cc_priority=True)),
        ("decomposition", N.tune_flags(ldd=1)),
    ])


@pytest.mark.parametrize("name", ["grid", "plain"])
def test_grid_and_plain_full_size_exact(name):
    f = shipped_flags(name)
    note(f"{name}: generate")
    g = gen.config(name)
    run_single(name, g, False, [("benchmarked", f | PROMISES), ("general contract", f), ("defaults", 0)])


@pytest.mark.parametrize("k", [2, 5, 10, 15, 20])
def test_knn_sweep_full_size_exact(k):
    f = shipped_flags(f"knn{k}")
    note(f"k-NN 2^22 points, k={k}: generate")
    g = gen.config(f"knn{k}")
    sets = [("benchmarked", f | PROMISES)]
    if k in (2, 20):
        sets.append(("defaults", 0))
    run_single(f"knn{k}", g, False, sets)


@pytest.mark.parametrize("name,tuned", [("sqr_torus_2000", "sqr_torus"), ("rec_torus_400", "rec_torus"),
                                        ("sqr_torus", "sqr_torus"), ("rec_torus", "rec_torus")])
def test_paper_tori_exact(name, tuned):
    """Percolated tori of the paper's SQR' / REC' shapes (p = 0.6), at the
    smaller sizes the oracle pins against Table 1 and at the full 10^8
    vertices the benchmark solves, with the tori's shipped flags."""
    f = shipped_flags(tuned)
    note(f"{name}: generate")
    g = gen.config(name)
    sets = [("benchmarked", f | PROMISES)]
    if name != tuned:
        sets.append(("defaults", 0))
    run_single(name, g, False, sets)


def test_batch4096_full_size_exact():
    """The 4096-graph batch in the benchmarked configuration (shipped flags,
    input promises; the general sequence alone and the split path the
    benchmark times), under the general contract and with the defaults."""
    f = shipped_flags("batch4096")
    note("batch of 4096: generate")
    u = gen.batch()
    vb = torch.from_numpy(u.vbegin).to(DEV)
    off = torch.from_numpy(u.offsets32()).to(DEV)
    adj = torch.from_numpy(u.adj).to(DEV)
    G = len(u.vbegin) - 1
    ws = alloc_workspace(u.n, u.num_arcs, G, DEV)
    outs = []
    for what, flags in (("benchmarked", f | PROMISES), ("general contract", f), ("defaults", 0)):
        note(f"batch of 4096: GPU batched solve ({what}) flags={flags:#x}")
        r = solve_batched(vb, off, adj, workspace=ws, flags=flags)
        assert read_device_status(ws) == 0, f"a device-side invariant check fired ({what})"
        outs.append((what, r.edge_label.cpu().numpy(), r.is_ap.cpu().numpy(), r.num_bcc.cpu().numpy()))
        del r
    del ws
    torch.cuda.empty_cache()
    # the benchmarked split: graphs of <= 3072 vertices packed onto the fused
    # kernels, the rest on the general sequence, each part a replayed HIP graph
    from paper_2301_01356_amd.batch import SplitBatchedSolver

    graphs = []
    for i in range(G):
        v0, v1 = int(u.vbegin[i]), int(u.vbegin[i + 1])
        a0, a1 = int(u.offsets[v0]), int(u.offsets[v1])
        graphs.append(gen.Csr(v1 - v0, u.offsets[v0 : v1 + 1] - a0, u.adj[a0:a1] - v0))
    note("batch of 4096: split path (fused small graphs + general sequence)")
    small_caps, big_caps = SplitBatchedSolver.capacities(graphs, N.SMALL_MAX_VERTICES)
    split = SplitBatchedSolver(small_caps, big_caps, device=DEV, flags=f | PROMISES)
    split.stage(graphs)
    split.launch()
    split.synchronize()
    split.replay()
    split.synchronize()
    sres = split.results()
    note("batch of 4096: oracle per graph")
    for i in range(G):
        v0, v1 = int(u.vbegin[i]), int(u.vbegin[i + 1])
        a0, a1 = int(u.offsets[v0]), int(u.offsets[v1])
        olab, oap, onb, _, _ = oracle.ht_bcc(u.offsets[v0 : v1 + 1] - a0, u.adj[a0:a1] - v0)
        for what, lab, ap, nb in outs:
            assert int(nb[i]) == onb, f"graph {i} ({what})"
            assert np.array_equal(ap[v0:v1], oap), f"graph {i} ({what})"
            assert np.array_equal(lab[a0:a1], olab), f"graph {i} ({what})"
        assert sres[i].num_bcc == onb, f"graph {i} (split path)"
        assert np.array_equal(sres[i].is_ap, oap), f"graph {i} (split path)"
        assert np.array_equal(sres[i].edge_label, olab), f"graph {i} (split path)"


def test_shipped_table_names_every_benchmark_workload():
    assert sorted(SHIPPED) == sorted(SHIP_WORKLOADS)
