"""GPU parity of the fused small-graph path (fastbcc_solve_small: one
workgroup per pack of consecutive graphs, all per-vertex state in LDS)
against the CPU oracle, graph by graph, and against the general batched
path.

Integer outputs: bit-exact canonical edge labels, AP flags and BCC counts.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2301_01356_amd import _native as N
from paper_2301_01356_amd import alloc_workspace, gen, read_device_status, solve_batched, solve_small
from paper_2301_01356_amd.api import greedy_packs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
MAXN = N.SMALL_MAX_VERTICES


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def shuffled_rows(g: gen.Csr, seed: int) -> gen.Csr:
    """Same graph, every row in a seeded random order (the fused path does
    not need sorted rows; labels are arc indices, so the oracle follows)."""
    rng = np.random.default_rng(seed)
    adj = g.adj.copy()
    for v in range(g.n):
        a, b = int(g.offsets[v]), int(g.offsets[v + 1])
        adj[a:b] = adj[a:b][rng.permutation(b - a)]
    return gen.Csr(g.n, g.offsets, adj)


def device_union(u: gen.Csr):
    return (torch.from_numpy(u.vbegin).to(DEV), torch.from_numpy(u.offsets32()).to(DEV),
            torch.from_numpy(u.adj).to(DEV))


def run_small(u: gen.Csr, flags=0, packs=None):
    vb, off, adj = device_union(u)
    pk = None if packs is None else torch.tensor(packs, dtype=torch.int32, device=DEV)
    r = solve_small(vb, off, adj, flags=flags, packs=pk)
    torch.cuda.synchronize()
    return r.edge_label.cpu().numpy(), r.is_ap.cpu().numpy(), r.num_bcc.cpu().numpy()


def check_union(graphs, u: gen.Csr, got, what: str, rejected=()):
    lab, ap, nb = got
    for i, g in enumerate(graphs):
        v0, v1 = int(u.vbegin[i]), int(u.vbegin[i + 1])
        a0, a1 = int(u.offsets[v0]), int(u.offsets[v1])
        if g.n > MAXN or i in rejected:
            assert nb[i] == -1, f"{what}: graph {i} (n={g.n}) above the limit got num_bcc {nb[i]}"
            continue
        olab, oap, onb, _, _ = oracle.ht_bcc(g.offsets, g.adj)
        if not np.array_equal(lab[a0:a1], olab):
            bad = np.flatnonzero(lab[a0:a1] != olab)
            pytest.fail(f"{what}: graph {i} (n={g.n}, arcs={g.num_arcs}): {bad.size} labels differ, first at "
                        f"arc {bad[0]}: gpu {lab[a0 + bad[0]]} oracle {olab[bad[0]]}")
        assert np.array_equal(ap[v0:v1], oap), f"{what}: graph {i} (n={g.n}) articulation points differ"
        assert nb[i] == onb, f"{what}: graph {i} (n={g.n}) num_bcc {nb[i]} != {onb}"


PARAM = {"random": 6.0, "lattice": 0.7, "knn": 5, "tree_back": 0.3}


def test_small_class_boundaries_every_family():
    """Sizes on both sides of each class boundary (256, 1024, the maximum)
    and just above it (rejected), every family, rows shuffled."""
    graphs = []
    for k, name in enumerate(gen.FAMILIES):
        for n in (1, 2, 3, 64, 255, 256, 257, 1023, 1024, 1025, 1535, 1536, 1537, MAXN - 1, MAXN, MAXN + 1):
            graphs.append(shuffled_rows(gen.family(name, n, PARAM[name], seed=100 * k + n), seed=n + k))
    u = gen.unite(graphs)
    note(f"boundaries: {len(graphs)} graphs, {u.n} vertices, {u.num_arcs} arcs")
    check_union(graphs, u, run_small(u), "class boundaries")


def test_small_mixed_stream_matches_oracle():
    """A few hundred graphs of the batched workload's mixed families, n
    log-uniform in [16, the maximum]."""
    graphs = [gen.mixed(21, i, 16, MAXN, 4.0, 16.0) for i in range(400)]
    u = gen.unite(graphs)
    note(f"mixed: {len(graphs)} graphs, {u.n} vertices, {u.num_arcs} arcs")
    check_union(graphs, u, run_small(u), "mixed stream")


def test_small_edge_cases():
    """Degenerate and adversarial shapes: empty graphs, isolated vertices,
    self-loops, parallel edges, a star (one vertex with every tree arc), a
    path and a cycle of the maximum size (longest tours), a clique, bridges
    between cycles."""
    n = MAXN
    star = gen.from_edges(n, [(0, v) for v in range(1, n)])
    path = gen.from_edges(n, [(v, v + 1) for v in range(n - 1)])
    cycle = gen.from_edges(n, [(v, (v + 1) % n) for v in range(n)])
    k = 70
    clique = gen.from_edges(k, [(i, j) for i in range(k) for j in range(i + 1, k)])
    loops = gen.multigraph_csr(6, [(0, 0), (0, 1), (0, 1), (1, 2), (2, 2), (2, 3), (3, 4), (4, 2), (5, 5)])
    para = gen.multigraph_csr(4, [(0, 1), (0, 1), (1, 2), (2, 3), (2, 3), (2, 3)])
    isolated = gen.multigraph_csr(5, [(1, 3)])
    empty = gen.Csr(0, np.zeros(1, np.int64), np.zeros(0, np.int32))
    lonely = gen.Csr(1, np.zeros(2, np.int64), np.zeros(0, np.int32))
    loop_only = gen.multigraph_csr(1, [(0, 0), (0, 0)])
    # cycles of 7 joined in a chain by bridges, plus a pendant path
    e = []
    for c in range(20):
        b = 7 * c
        e += [(b + i, b + (i + 1) % 7) for i in range(7)]
        if c:
            e.append((b - 7, b))
    e += [(140 + i, 141 + i) for i in range(9)] + [(3, 140)]
    chain = gen.from_edges(150, e)
    graphs = [empty, star, lonely, path, loops, cycle, empty, clique, para, isolated, loop_only, chain,
              shuffled_rows(star, 5), shuffled_rows(cycle, 6), empty]
    u = gen.unite(graphs)
    note(f"edge cases: {len(graphs)} graphs, {u.n} vertices, {u.num_arcs} arcs")
    check_union(graphs, u, run_small(u), "edge cases")


def test_small_single_graph_and_flags():
    """One graph alone (one workgroup in the last class), with the input
    promise flags accepted."""
    g = gen.family("lattice", MAXN, 0.8, seed=3)
    u = gen.unite([g])
    note("single lattice graph, promise flags")
    check_union([g], u, run_small(u, flags=N.FLAG_SORTED_ROWS | N.FLAG_NO_SELF_LOOPS), "single graph")


def test_small_agrees_with_general_batched_path():
    """The fused path and the general batched path give the same labels on
    the small graphs of the batched workload's recipe."""
    u = gen.batch(seed=31, count=600, nmin=64, nmax=MAXN)
    note(f"fused vs general: {u.vbegin.size - 1} graphs, {u.n} vertices")
    vb, off, adj = device_union(u)
    G = vb.numel() - 1
    r1 = solve_small(vb, off, adj)
    ws = alloc_workspace(u.n, u.num_arcs, G, DEV)
    r2 = solve_batched(vb, off, adj, workspace=ws)
    assert read_device_status(ws) == 0
    torch.cuda.synchronize()
    assert torch.equal(r1.num_bcc, r2.num_bcc)
    assert torch.equal(r1.is_ap, r2.is_ap)
    assert torch.equal(r1.edge_label, r2.edge_label)


def test_small_hip_graph_replays():
    """Captured into a HIP graph and replayed: every replay, with eager work
    and synchronisation between replays, equals the eager result."""
    graphs = [gen.mixed(41, i, 16, MAXN, 4.0, 16.0) for i in range(120)]
    u = gen.unite(graphs)
    vb, off, adj = device_union(u)
    eager = solve_small(vb, off, adj)
    torch.cuda.synchronize()
    out = solve_small(vb, off, adj)  # output buffers the graph writes
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        solve_small(vb, off, adj, out=out, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        note(f"replay {rep}")
        out.edge_label.fill_(-7)
        out.is_ap.fill_(9)
        out.num_bcc.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out.edge_label, eager.edge_label), f"replay {rep}: labels differ"
        assert torch.equal(out.is_ap, eager.is_ap), f"replay {rep}: AP flags differ"
        assert torch.equal(out.num_bcc, eager.num_bcc), f"replay {rep}: counts differ"
    check_union(graphs, u, (eager.edge_label.cpu().numpy(), eager.is_ap.cpu().numpy(),
                            eager.num_bcc.cpu().numpy()), "eager before capture")


@pytest.mark.parametrize("capacity", [256, 1024, MAXN])
def test_small_packs_match_oracle(capacity):
    """Consecutive graphs packed into one workgroup's union (greedy packs of
    at most `capacity` vertices; bigger graphs alone), empty graphs inside
    packs, rows shuffled: every graph's own labels, flags and count."""
    empty = gen.Csr(0, np.zeros(1, np.int64), np.zeros(0, np.int32))
    graphs = []
    for i in range(300):
        graphs.append(shuffled_rows(gen.mixed(51, i, 2, MAXN, 4.0, 16.0), seed=i))
        if i % 37 == 0:
            graphs += [empty, empty]
    u = gen.unite(graphs)
    packs = greedy_packs([g.n for g in graphs], capacity)
    note(f"packs of <= {capacity}: {len(graphs)} graphs in {len(packs) - 1} packs")
    check_union(graphs, u, run_small(u, packs=packs), f"packs of {capacity}")


def test_small_pack_limits():
    """A pack above the vertex limit, or holding more graphs than the limit,
    is refused as a whole (num_bcc -1); the packs around it are solved."""
    a = gen.family("random", 2000, 6.0, seed=1)
    b = gen.family("lattice", 1500, 0.7, seed=2)
    c = gen.family("knn", 700, 5, seed=3)
    empty = gen.Csr(0, np.zeros(1, np.int64), np.zeros(0, np.int32))
    graphs = [c, a, b, c] + [empty] * (MAXN + 1) + [c]
    u = gen.unite(graphs)
    k = 4 + MAXN + 1
    packs = [0, 1, 3, 4, k, k + 1]  # [c] [a b]: 3500 vertices [c] [empties] [c]
    note("pack limits")
    lab, ap, nb = run_small(u, packs=packs)
    assert nb[1] == -1 and nb[2] == -1, "a pack above the vertex limit must be refused"
    assert (nb[4:k] == -1).all(), "a pack with more graphs than the limit must be refused"
    check_union(graphs, u, (lab, ap, nb), "pack limits", rejected=set([1, 2]) | set(range(4, k)))


def test_small_packed_agrees_with_general_batched_path():
    """Tiny graphs (the regime packing is for): packed fused path == general
    batched path on every output."""
    u = gen.batch(seed=32, count=3000, nmin=2, nmax=400)
    G = u.vbegin.size - 1
    note(f"packed tiny graphs: {G} graphs, {u.n} vertices")
    vb, off, adj = device_union(u)
    pk = torch.tensor(greedy_packs(np.diff(u.vbegin), MAXN), dtype=torch.int32, device=DEV)
    r1 = solve_small(vb, off, adj, packs=pk)
    ws = alloc_workspace(u.n, u.num_arcs, G, DEV)
    r2 = solve_batched(vb, off, adj, workspace=ws)
    assert read_device_status(ws) == 0
    torch.cuda.synchronize()
    assert torch.equal(r1.num_bcc, r2.num_bcc)
    assert torch.equal(r1.is_ap, r2.is_ap)
    assert torch.equal(r1.edge_label, r2.edge_label)


def test_split_batched_solver_two_batches():
    """The batch layer's split path (small graphs packed onto the fused
    kernels, the rest on the general sequence, two streams, each part
    replayed from its own HIP graph): two batches in a row, the second with
    fewer and other graphs, every result equal to the oracle's."""
    from paper_2301_01356_amd.batch import SplitBatchedSolver

    first = [gen.mixed(61, i, 16, 8192, 4.0, 16.0) for i in range(160)]
    second = [gen.mixed(62, i, 2, 6000, 4.0, 16.0) for i in range(90)]
    caps = [SplitBatchedSolver.capacities(b, MAXN) for b in (first, second)]
    small_caps = tuple(max(c[0][k] for c in caps) for k in range(3))
    big_caps = tuple(max(c[1][k] for c in caps) for k in range(3))
    solver = SplitBatchedSolver(small_caps, big_caps, small_max=MAXN, device=DEV)
    for what, graphs in (("first", first), ("second", second)):
        note(f"split solver, {what} batch: {len(graphs)} graphs")
        res = solver.solve(graphs)
        for i, (g, r) in enumerate(zip(graphs, res)):
            olab, oap, onb, _, _ = oracle.ht_bcc(g.offsets, g.adj)
            assert r.num_bcc == onb, f"{what} batch graph {i} (n={g.n}): num_bcc {r.num_bcc} != {onb}"
            assert np.array_equal(r.is_ap, oap), f"{what} batch graph {i} (n={g.n}): AP flags differ"
            assert np.array_equal(r.edge_label, olab), f"{what} batch graph {i} (n={g.n}): labels differ"
