"""GPU tests of the batched (HIP-graph replay) and serving paths."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2301_01356_amd import gen, solve
from paper_2301_01356_amd.batch import BatchedSolver
from paper_2301_01356_amd.serve import Request, Server, hip_slots, latency_summary, poisson_arrivals

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def check_oracle(g, lab, ap, nb, what):
    olab, oap, onb, _, _ = oracle.ht_bcc(g.offsets, g.adj)
    assert np.array_equal(lab, olab), f"{what}: labels differ"
    assert np.array_equal(ap, oap), f"{what}: articulation points differ"
    assert nb == onb, f"{what}: num_bcc {nb} != {onb}"


def test_graph_replay_matches_oracle_across_batches():
    batch_a = [gen.mixed(51, i, 8, 2500, 4.0, 16.0) for i in range(24)]
    batch_b = [gen.mixed(52, i, 8, 4000, 4.0, 16.0) for i in range(9)]
    cap_v = 1 + max(sum(g.n for g in batch_a), sum(g.n for g in batch_b)) + 100
    cap_a = max(sum(g.num_arcs for g in batch_a), sum(g.num_arcs for g in batch_b)) + 1000
    s = BatchedSolver(cap_v, cap_a, 32, device=DEV, use_graph=True)
    for rnd, batch in enumerate([batch_a, batch_b, batch_a, batch_b, batch_a]):
        note(f"replay {rnd}: {len(batch)} graphs")
        res = s.solve(batch)
        assert s.graph is not None
        # the program's own eager work between replays
        x = torch.arange(1 << 20, device=DEV, dtype=torch.int64).sum().item()
        assert x == (1 << 20) * ((1 << 20) - 1) // 2
        torch.cuda.synchronize()
        for i, (g, r) in enumerate(zip(batch, res)):
            check_oracle(g, r.edge_label, r.is_ap, r.num_bcc, f"replay {rnd} graph {i}")


def test_graph_replay_equals_eager():
    batch = [gen.mixed(53, i, 8, 3000, 4.0, 16.0) for i in range(16)]
    cap_v = sum(g.n for g in batch) + 64
    cap_a = sum(g.num_arcs for g in batch) + 64
    note("eager vs graph")
    eager = BatchedSolver(cap_v, cap_a, 16, device=DEV, use_graph=False).solve(batch)
    graph_s = BatchedSolver(cap_v, cap_a, 16, device=DEV, use_graph=True)
    for rep in range(3):
        got = graph_s.solve(batch)
        for e, g in zip(eager, got):
            assert np.array_equal(e.edge_label, g.edge_label) and np.array_equal(e.is_ap, g.is_ap)
            assert e.num_bcc == g.num_bcc


def test_fixed_shape_buffers_hold_the_padded_union():
    """After staging, the device buffers of the fixed-shape solver equal the
    host-side padded union (graph-local ids made global on the device), for
    graphs staged through pinned staging and graphs already pinned."""
    from paper_2301_01356_amd.batch import PinnedGraph, pack

    graphs = [gen.mixed(57, i, 8, 900, 4.0, 16.0) for i in range(10)]
    mixed = [PinnedGraph(g) if i % 3 == 1 else g for i, g in enumerate(graphs)]
    cap_v = sum(g.n for g in graphs) + 9
    cap_a = sum(g.num_arcs for g in graphs) + 31
    s = BatchedSolver(cap_v, cap_a, 12, device=DEV, use_graph=False)
    s.stage(mixed)
    s._copy_in()
    s.stream.synchronize()
    vb, off, adj, _ = pack(graphs, cap_v, cap_a, 12)
    note("fixed-shape buffers vs pack()")
    assert np.array_equal(s.d_vbegin.cpu().numpy(), vb)
    assert np.array_equal(s.d_off.cpu().numpy(), off)
    assert np.array_equal(s.d_adj.cpu().numpy(), adj)


def test_serving_each_result_same_alone_and_in_the_mix():
    """Served with the benchmark's serving flags (general input contract,
    shipped mixed-batch tuning) and live free-HBM admission: every result
    equals the request's plain solve alone (labels, AP flags, count and
    device digest), every fifth one the oracle too."""
    from paper_2301_01356_amd.batch import PinnedGraph
    from paper_2301_01356_amd.serve import PlainSlot, serving_flags

    count = 40
    reqs = []
    arr = poisson_arrivals(count, 400.0, 5)
    for i in range(count):
        g = gen.mixed(55, i, 64, 60000, 4.0, 32.0)
        reqs.append(Request(i, PinnedGraph(g) if i % 2 else g, float(arr[i])))
    flags = serving_flags()
    slots = hip_slots(3, cap_v=200000, cap_a=4_000_000, cap_g=16, device=DEV, flags=flags, digests=True)
    srv = Server(slots, hbm_budget=8 << 30, free_hbm=lambda: torch.cuda.mem_get_info()[0])
    note(f"serving {count} requests on {len(slots)} slots, flags {flags:#x}")
    comps = srv.run(reqs)
    assert srv.stats["batches"] < count  # requests were batched together
    assert srv.stats["budget_reads"] >= srv.stats["batches"]
    serial = Server([PlainSlot(60001, 4_000_000, DEV, flags, digests=True)], hbm_budget=8 << 30, max_batch_graphs=1)
    note("serial plain solves of the same requests")
    comps1 = serial.run(reqs)
    for r, c, c1 in zip(reqs, comps, comps1):
        assert c.ok and c1.ok, (c.error, c1.error)
        off = torch.from_numpy(np.asarray(r.graph.offsets, np.int32)).to(DEV)
        adj = torch.from_numpy(np.asarray(r.graph.adj, np.int32)).to(DEV)
        alone = solve(off, adj, flags=flags)
        torch.cuda.synchronize()
        assert np.array_equal(alone.edge_label.cpu().numpy(), c.edge_label), f"request {r.rid}: labels differ"
        assert np.array_equal(alone.is_ap.cpu().numpy(), c.is_ap), f"request {r.rid}: APs differ"
        assert int(alone.num_bcc.item()) == c.num_bcc
        assert np.array_equal(c1.edge_label, c.edge_label) and c1.digest == c.digest and c1.num_bcc == c.num_bcc
        if r.rid % 5 == 0:
            check_oracle(r.graph, c.edge_label, c.is_ap, c.num_bcc, f"request {r.rid}")
    s = latency_summary(comps)
    note(f"p50 {s['p50_ms']:.2f} ms p99 {s['p99_ms']:.2f} ms")


def test_serving_general_contract_unsorted_rows_and_self_loops():
    """Serving does not trust the sorted-row and loop-free promises: requests
    with shuffled rows and self-loops are served correctly (oracle)."""
    from paper_2301_01356_amd.serve import serving_flags

    rng = np.random.default_rng(23)
    reqs = []
    for i in range(12):
        n = int(rng.integers(5, 400))
        edges = [(int(rng.integers(0, n)), int(rng.integers(0, n))) for _ in range(int(rng.integers(n, 4 * n)))]
        g = gen.multigraph_csr(n, edges)
        adj = g.adj.copy()
        for v in range(n):
            a, b = g.offsets[v], g.offsets[v + 1]
            adj[a:b] = rng.permutation(adj[a:b])
        reqs.append(Request(i, gen.Csr(n, g.offsets, adj), 0.0))
    slots = hip_slots(2, cap_v=5000, cap_a=40000, cap_g=8, device=DEV, flags=serving_flags())
    note("serving unsorted rows with self-loops")
    comps = Server(slots, hbm_budget=1 << 30).run(reqs)
    for r, c in zip(reqs, comps):
        assert c.ok, c.error
        check_oracle(r.graph, c.edge_label, c.is_ap, c.num_bcc, f"request {r.rid}")


def _corrupt_batch():
    """A batch of valid graphs, then damage inside some of them (the batch
    layout -- graph ranges and each graph's first row start -- stays valid)."""
    graphs = [gen.mixed(81, i, 20, 600, 4.0, 12.0) for i in range(8)]
    u = gen.unite(graphs)
    off = u.offsets.astype(np.int32).copy()
    adj = u.adj.copy()
    vb = u.vbegin

    def arcs(g):
        return int(off[vb[g]]), int(off[vb[g + 1]])

    a0, _ = arcs(1)
    adj[a0 + 3] = int(vb[2]) + 1  # graph 1: an arc into graph 2
    v = int(vb[3]) + 2
    off[v], off[v + 1] = off[v + 1], off[v]  # graph 3: decreasing offsets
    if off[v] == off[v + 1]:
        off[v] += 1
    a0, _ = arcs(4)
    adj[a0] = -5  # graph 4: a negative id
    off[int(vb[5]) + 1] = len(adj)  # graph 5: a row that runs past the graph's arcs
    return graphs, u, off, adj, {1, 3, 4, 5}


def test_device_input_check_finds_and_repairs_damaged_graphs():
    from paper_2301_01356_amd import check_batched, solve_batched
    from paper_2301_01356_amd import _native as N

    graphs, u, off, adj, bad = _corrupt_batch()
    G = len(graphs)
    d_vb = torch.from_numpy(u.vbegin).to(DEV)
    d_off = torch.from_numpy(off).to(DEV)
    d_adj = torch.from_numpy(adj).to(DEV)
    note("device input check, no repair")
    st = check_batched(d_off, d_adj, d_vb).cpu().numpy()
    assert {i for i in range(G) if st[i]} == bad
    assert np.all(st[list(bad)] == N.ERR_INVALID_GRAPH)
    assert np.array_equal(d_off.cpu().numpy(), off) and np.array_equal(d_adj.cpu().numpy(), adj)  # untouched
    note("device input check with repair, then a batched solve of the whole batch")
    st = check_batched(d_off, d_adj, d_vb, repair=True).cpu().numpy()
    assert {i for i in range(G) if st[i]} == bad
    roff, radj = d_off.cpu().numpy(), d_adj.cpu().numpy()
    for g in range(G):
        v0, v1 = int(u.vbegin[g]), int(u.vbegin[g + 1])
        a0, a1 = int(u.offsets[v0]), int(u.offsets[v1])
        if g in bad:  # every arc a self-loop of the first vertex, other rows empty
            assert np.all(radj[a0:a1] == v0) and np.all(roff[v0 + 1 : v1 + 1] == a1) and roff[v0] == a0
        else:
            assert np.array_equal(roff[v0:v1], off[v0:v1]) and np.array_equal(radj[a0:a1], adj[a0:a1])
    r = solve_batched(d_vb, d_off, d_adj)
    torch.cuda.synchronize()
    lab, ap, nb = r.edge_label.cpu().numpy(), r.is_ap.cpu().numpy(), r.num_bcc.cpu().numpy()
    for g in set(range(G)) - bad:
        v0, v1 = int(u.vbegin[g]), int(u.vbegin[g + 1])
        a0, a1 = int(u.offsets[v0]), int(u.offsets[v1])
        check_oracle(graphs[g], lab[a0:a1], ap[v0:v1], int(nb[g]), f"graph {g}")


def test_device_input_check_of_the_promises_and_symmetry():
    from paper_2301_01356_amd import check_batched
    from paper_2301_01356_amd import _native as N

    good = gen.from_edges(6, [(0, 1), (1, 2), (2, 0), (2, 3), (3, 4), (4, 5), (5, 3)])
    unsorted = gen.Csr(good.n, good.offsets, good.adj.copy())
    r0, r1 = int(unsorted.offsets[2]), int(unsorted.offsets[3])
    unsorted.adj[r0:r1] = unsorted.adj[r0:r1][::-1]
    loopy = gen.multigraph_csr(4, [(0, 1), (1, 2), (2, 2), (2, 3)])
    asym = gen.Csr(good.n, good.offsets, good.adj.copy())
    asym.adj[int(asym.offsets[4])] = 2  # 4 -> 2 without 2 -> 4 (row 4 stays sorted: 2 < 5)
    graphs = [good, unsorted, loopy, asym]
    u = gen.unite(graphs)
    d_vb = torch.from_numpy(u.vbegin).to(DEV)
    d_off = torch.from_numpy(u.offsets.astype(np.int32)).to(DEV)
    d_adj = torch.from_numpy(u.adj).to(DEV)
    note("device input check: sorted rows, loops, symmetry")
    st = lambda f: check_batched(d_off, d_adj, d_vb, flags=f).cpu().numpy().tolist()
    assert st(0) == [0, 0, 0, 0]
    assert st(N.FLAG_SORTED_ROWS) == [0, 5, 0, 0]
    assert st(N.FLAG_NO_SELF_LOOPS) == [0, 0, 5, 0]
    assert st(N.FLAG_SORTED_ROWS | N.FLAG_VALIDATE) == [0, 5, 0, 5]


def test_serving_rejects_damaged_requests_and_serves_the_rest():
    from paper_2301_01356_amd.serve import PlainSlot, serving_flags

    reqs = []
    for i in range(16):
        g = gen.mixed(83, i, 30, 3000, 4.0, 16.0)
        if i % 4 == 1:  # an id beyond the graph
            adj = g.adj.copy()
            adj[len(adj) // 2] = g.n + 7
            g = gen.Csr(g.n, g.offsets, adj)
        elif i % 4 == 3:  # decreasing offsets inside the graph
            off = g.offsets.copy()
            v = g.n // 2
            off[v], off[v + 1] = off[v + 1] + 1, off[v]
            g = gen.Csr(g.n, off, g.adj)
        reqs.append(Request(i, g, 0.0))
    flags = serving_flags()
    for name, slots, mb in (("served", hip_slots(2, 60000, 600000, 8, device=DEV, flags=flags), None),
                            ("serial", [PlainSlot(3001, 600000, DEV, flags)], 1)):
        note(f"{name}: damaged requests among good ones")
        comps = Server(slots, hbm_budget=1 << 30, max_batch_graphs=mb).run(reqs)
        for r, c in zip(reqs, comps):
            if r.rid % 4 in (1, 3):
                assert not c.ok and "invalid graph" in c.error, (name, r.rid)
            else:
                assert c.ok, (name, r.rid, c.error)
                check_oracle(r.graph, c.edge_label, c.is_ap, c.num_bcc, f"{name} request {r.rid}")
