"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

All outputs are integers, so the bar is bit-exact equality of the canonical
edge labels, the articulation-point flags and the BCC count.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2301_01356_amd import _native as N
from paper_2301_01356_amd import alloc_workspace, gen, read_device_status, solve
from paper_2301_01356_amd import solve_batched as _solve_batched
from paper_2301_01356_amd.api import BccResult

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def to_dev(g, off64=False):
    off = torch.from_numpy(g.offsets if off64 else g.offsets32()).to(DEV)
    adj = torch.from_numpy(g.adj).to(DEV)
    return off, adj


def gpu_solve(g, off64=False, flags=0):
    """Solve through the C ABI; the device status word (the solve's in-kernel
    invariant checks) must read 0 afterwards."""
    off, adj = to_dev(g, off64)
    ws = alloc_workspace(g.n, g.num_arcs, 1, DEV)
    r = solve(off, adj, workspace=ws, flags=flags)
    assert read_device_status(ws) == 0, "a device-side invariant check fired"
    return r.edge_label.cpu().numpy(), r.is_ap.cpu().numpy(), int(r.num_bcc.item())


def solve_batched(vb, off, adj, flags=0, workspace=None):
    """Batched solve through the C ABI with the device status checked."""
    ws = workspace if workspace is not None else alloc_workspace(off.numel() - 1, adj.numel(), vb.numel() - 1, DEV)
    r = _solve_batched(vb, off, adj, workspace=ws, flags=flags)
    st = read_device_status(ws)
    assert st == 0, f"a device-side invariant check fired ({st})"
    return r


def assert_parity(g, got, what=""):
    lab, ap, nb, _, _ = oracle.ht_bcc(g.offsets, g.adj)
    glab, gap, gnb = got
    if not np.array_equal(glab, lab):
        bad = np.flatnonzero(glab != lab)
        pytest.fail(f"{what}: {bad.size} edge labels differ, first at arc {bad[0]}: gpu {glab[bad[0]]} oracle {lab[bad[0]]}")
    assert np.array_equal(gap, ap), f"{what}: articulation points differ at {np.flatnonzero(gap != ap)[:10]}"
    assert gnb == nb, f"{what}: num_bcc {gnb} != {nb}"


SMALL = ["plain_small", "grid_small", "rmat_small", "batch_small"]


@pytest.mark.parametrize("name", SMALL)
@pytest.mark.parametrize("off64", [False, True])
def test_small_configs(name, off64):
    note(f"{name} off64={off64}")
    g = gen.config(name)
    assert_parity(g, gpu_solve(g, off64), name)


SORTED_FLAGS = [
    N.FLAG_SORTED_ROWS,
    N.FLAG_SORTED_ROWS | N.FLAG_NO_SELF_LOOPS | N.tune_flags(sampled_tags=True, free_first_round=True, lcc_rounds=0),
    N.FLAG_SORTED_ROWS | N.tune_flags(lcc_priority=True, sampled_tags=True),
    N.FLAG_SORTED_ROWS | N.tune_flags(sampled_tags=True),
    N.FLAG_SORTED_ROWS | N.tune_flags(sampled_tags=True, cc_priority=True, ruler_shift=7, tile_shift=4),
    N.FLAG_SORTED_ROWS | N.tune_flags(ldd=1, sample_rounds=0),
]


@pytest.mark.parametrize("name", SMALL)
@pytest.mark.parametrize("flags", SORTED_FLAGS)
def test_sorted_row_read_out(name, flags):
    """The mirror read-out (sorted rows) against the oracle, alone and with
    the other tuning variants."""
    note(f"{name} flags={flags:#x}")
    g = gen.config(name)
    assert_parity(g, gpu_solve(g, flags=flags), f"{name} {flags:#x}")


@pytest.mark.parametrize("flags", SORTED_FLAGS[:1] + SORTED_FLAGS[2:3])
def test_sorted_row_read_out_multigraphs(flags):
    """Sorted multigraphs with self-loops: copies of an edge to a head are
    mirrored together."""
    rng = np.random.default_rng(11)
    for t in range(40):
        n = int(rng.integers(2, 60))
        m = int(rng.integers(0, 3 * n))
        edges = [(int(rng.integers(0, n)), int(rng.integers(0, n))) for _ in range(m)]
        edges += edges[: int(rng.integers(0, 6))]
        edges += [(i, i + 1) for i in range(0, n - 1, 3)]  # pendant paths and bridges
        g = gen.multigraph_csr(n, edges)
        for v in range(n):
            row = g.adj[g.offsets[v] : g.offsets[v + 1]]
            assert np.all(row[1:] >= row[:-1]), "generator rows must be sorted"
        note(f"sorted multigraph #{t} n={n} arcs={g.num_arcs} flags={flags:#x}")
        assert_parity(g, gpu_solve(g, flags=flags), f"sorted multigraph {t}")


def sparse_rows_graph(seed, n, isolated, hubs):
    """Loop-free graph whose rows are mostly empty or short, with runs of
    more than 64 empty rows and a few hubs: 64-arc windows then span from
    one row to well over 64 rows."""
    rng = np.random.default_rng(seed)
    live = np.flatnonzero(rng.random(n) >= isolated)
    live = live[(live < n // 3) | (live > n // 3 + 300)]  # a run of empty rows
    edges = []
    for i in range(0, len(live) - 1, 2):  # a matching: rows of degree 1
        edges.append((int(live[i]), int(live[i + 1])))
    for i in range(0, len(live) - 2, 7):  # short paths and triangles
        edges.append((int(live[i]), int(live[i + 2])))
    for h in live[rng.choice(len(live), size=hubs, replace=False)]:
        for v in rng.choice(live, size=min(len(live), 700), replace=False):
            if int(v) != int(h):
                edges.append((int(h), int(v)))
    return gen.from_edges(n, edges)


ROW_FILL_FLAGS = [
    N.FLAG_SORTED_ROWS | N.FLAG_NO_SELF_LOOPS | N.tune_flags(tile_shift=t)
    for t in (2, 4, 6)
] + [N.FLAG_SORTED_ROWS | N.FLAG_NO_SELF_LOOPS | N.tune_flags(sampled_tags=True, free_first_round=True)]


@pytest.mark.parametrize("flags", ROW_FILL_FLAGS)
@pytest.mark.parametrize("shape", [(1, 3000, 0.9, 0), (2, 20000, 0.6, 3), (3, 50000, 0.97, 2), (4, 777, 0.0, 1)])
def test_loop_free_row_fill(flags, shape):
    """The row-wise label fill for loop-free sorted rows: windows inside one
    row, windows over a few rows, windows over more than 64 rows and runs of
    empty rows between windows, at several tile sizes."""
    seed, n, isolated, hubs = shape
    g = sparse_rows_graph(seed, n, isolated, hubs)
    note(f"sparse rows seed={seed} n={n} arcs={g.num_arcs} flags={flags:#x}")
    assert_parity(g, gpu_solve(g, flags=flags), f"sparse rows {shape} {flags:#x}")


@pytest.mark.parametrize("shift", [0, 1, 2, 3])
def test_loop_free_row_fill_label_alignment(shift):
    """The fill stores four labels at once where the label buffer is 16-byte
    aligned; a buffer at 4, 8 or 12 bytes past that takes the one-label
    stores.  Both give the oracle's labels."""
    g = gen.config("rmat_small")
    off, adj = to_dev(g)
    A, n = g.num_arcs, g.n
    buf = torch.full((A + 4,), -9, dtype=torch.int32, device=DEV)
    out = BccResult(buf[shift : shift + A], torch.empty(n, dtype=torch.uint8, device=DEV),
                    torch.empty(1, dtype=torch.int64, device=DEV))
    note(f"rmat_small label buffer offset {4 * shift} bytes")
    flags = N.FLAG_SORTED_ROWS | N.FLAG_NO_SELF_LOOPS | N.tune_flags(sampled_tags=True)
    solve(off, adj, out=out, flags=flags)
    torch.cuda.synchronize()
    got = (out.edge_label.cpu().numpy(), out.is_ap.cpu().numpy(), int(out.num_bcc.item()))
    assert_parity(g, got, f"label offset {shift}")
    rest = torch.cat([buf[:shift], buf[shift + A :]]).cpu().numpy()
    assert np.all(rest == -9), "the solve wrote outside the label buffer"


def cycle(n):
    return [(i, (i + 1) % n) for i in range(n)]


def path(n):
    return [(i, i + 1) for i in range(n - 1)]


CLOSED = {
    "cycle3": (3, cycle(3)),
    "cycle1000": (1000, cycle(1000)),
    "path2": (2, path(2)),
    "path5000": (5000, path(5000)),
    "star": (65, [(0, i) for i in range(1, 65)]),
    "k7": (7, [(i, j) for i in range(7) for j in range(i + 1, 7)]),
    "two_cycles": (8, cycle(5) + [(0, 5), (5, 6), (6, 7), (7, 0)]),
    "isolated_plus_edge": (6, [(1, 2)]),
    "single_vertex": (1, []),
}


@pytest.mark.parametrize("name", sorted(CLOSED))
def test_closed_forms(name):
    n, e = CLOSED[name]
    note(name)
    g = gen.from_edges(n, e) if e else gen.Csr(n, np.zeros(n + 1, np.int64), np.zeros(0, np.int32))
    assert_parity(g, gpu_solve(g), name)


def test_open_grid_and_long_path():
    note("grid 64x80 p=1 + path 3000")
    g = gen.grid(seed=5, rows=64, cols=80, p=1.0, path_len=3000, chord_block=100)
    assert_parity(g, gpu_solve(g), "grid+path")


@pytest.mark.parametrize("ruler_shift", [3, 4])
@pytest.mark.parametrize("what", ["rmat19", "path", "forest"])
def test_two_level_list_ranking(what, ruler_shift):
    """Euler tours long enough for the second ruling level (at least 2^16
    rulers): a power-law graph, one long path, and many path trees."""
    if what == "rmat19":
        g = gen.rmat(seed=7, scale=19, edge_factor=4)
    elif what == "path":
        g = gen.from_edges(600_000, path(600_000))
    else:
        edges = [(i, i + 1) for i in range(700_000) if i % 997 != 996]
        g = gen.from_edges(700_001, edges)
    flags = N.tune_flags(ruler_shift=ruler_shift)
    note(f"two-level list ranking {what} n={g.n} arcs={g.num_arcs} flags={flags:#x}")
    assert_parity(g, gpu_solve(g, flags=flags), f"{what} ruler {ruler_shift}")


def test_multigraph_self_loops_unsorted_rows():
    rng = np.random.default_rng(3)
    for t in range(60):
        n = int(rng.integers(1, 40))
        m = int(rng.integers(0, 80))
        edges = [(int(rng.integers(0, n)), int(rng.integers(0, n))) for _ in range(m)]
        edges += edges[: int(rng.integers(0, 5))]
        g = gen.multigraph_csr(n, edges)
        adj = g.adj.copy()
        for v in range(n):
            s, e = g.offsets[v], g.offsets[v + 1]
            adj[s:e] = rng.permutation(adj[s:e])
        g = gen.Csr(n, g.offsets, adj)
        note(f"multigraph #{t} n={n} arcs={g.num_arcs}")
        assert_parity(g, gpu_solve(g), f"multigraph {t}")


@pytest.mark.parametrize("flags", [
    N.tune_flags(ruler_shift=3), N.tune_flags(ruler_shift=10), N.tune_flags(sample_rounds=0),
    N.tune_flags(sample_rounds=1), N.tune_flags(tile_shift=6), N.tune_flags(ruler_shift=7, tile_shift=3),
    N.tune_flags(cc_priority=True), N.tune_flags(cc_priority=True, sample_rounds=0),
    N.tune_flags(ldd=1), N.tune_flags(ldd=3, sample_rounds=0), N.tune_flags(ldd=2, cc_priority=True),
    N.tune_flags(sampled_tags=True), N.tune_flags(sampled_tags=True, cc_priority=True, tile_shift=3),
    N.tune_flags(sampled_tags=True, ldd=1, sample_rounds=0),
    N.tune_flags(sampled_tags=True, tag_samples=2), N.tune_flags(sampled_tags=True, tag_samples=1),
    N.tune_flags(free_first_round=True), N.tune_flags(free_first_round=True, cc_priority=True, sample_rounds=1),
    N.tune_flags(lcc_priority=True), N.tune_flags(lcc_priority=True, sampled_tags=True, sample_rounds=0),
    N.tune_flags(lcc_rounds=0), N.tune_flags(lcc_rounds=1, lcc_priority=True, sampled_tags=True),
    N.tune_flags(vertex_block=64), N.tune_flags(vertex_block=128, cc_priority=True, free_first_round=True),
    N.tune_flags(vertex_block=512, sampled_tags=True, tag_samples=1, lcc_priority=True),
    N.tune_flags(free_first_round=True, compress_free_round=True, cc_priority=True),
    N.tune_flags(free_first_round=True, compress_free_round=True, sample_rounds=1),
    N.tune_flags(xcd_order=True), N.tune_flags(xcd_order=True, vertex_block=64, sampled_tags=True, cc_priority=True),
    N.tune_flags(xcd_order=True, lcc_priority=True, free_first_round=True, lcc_rounds=1, vertex_block=512),
])
@pytest.mark.parametrize("cfg", ["rmat_small", "grid_small"])
def test_tuning_fields_never_change_results(flags, cfg):
    note(f"{cfg} flags={flags:#x}")
    g = gen.config(cfg)
    assert_parity(g, gpu_solve(g, flags=flags), f"flags {flags:#x}")


def test_repeated_solves_identical():
    g = gen.config("grid_small")
    note("grid_small x5")
    first = gpu_solve(g)
    for _ in range(4):
        again = gpu_solve(g)
        assert np.array_equal(first[0], again[0]) and np.array_equal(first[1], again[1]) and first[2] == again[2]


BATCH_FLAGS = [0, N.FLAG_SORTED_ROWS | N.FLAG_NO_SELF_LOOPS | N.tune_flags(sampled_tags=True, free_first_round=True,
                                                                          ruler_shift=3),
               N.tune_flags(xcd_order=True, cc_priority=True, lcc_priority=True, free_first_round=True),
               N.tune_flags(graph_cc=True),
               N.FLAG_SORTED_ROWS | N.FLAG_NO_SELF_LOOPS | N.tune_flags(graph_cc=True, sampled_tags=True,
                                                                          lcc_priority=True, ruler_shift=3)]


@pytest.mark.parametrize("flags", BATCH_FLAGS)
def test_batched_equals_each_graph_alone(flags):
    rng = np.random.default_rng(9)
    graphs = [gen.mixed(41, i, 8, 3000, 4.0, 16.0) for i in range(40)]
    graphs.append(gen.Csr(3, np.zeros(4, np.int64), np.zeros(0, np.int32)))  # an edgeless graph
    graphs.insert(5, gen.from_edges(4, cycle(4)))
    empty = gen.Csr(0, np.zeros(1, np.int64), np.zeros(0, np.int32))  # no vertices at all
    graphs = [empty] + graphs[:20] + [empty, empty] + graphs[20:] + [empty]
    u = gen.unite(graphs)
    note(f"batched {len(graphs)} graphs n={u.n} arcs={u.num_arcs} flags={flags:#x}")
    vb = torch.from_numpy(u.vbegin).to(DEV)
    off, adj = to_dev(u)
    r = solve_batched(vb, off, adj, flags=flags)
    torch.cuda.synchronize()
    lab = r.edge_label.cpu().numpy()
    ap = r.is_ap.cpu().numpy()
    nb = r.num_bcc.cpu().numpy()
    for i, g in enumerate(graphs):
        a0, a1 = u.offsets[u.vbegin[i]], u.offsets[u.vbegin[i + 1]]
        got = (lab[a0:a1], ap[u.vbegin[i] : u.vbegin[i + 1]], int(nb[i]))
        assert_parity(g, got, f"graph {i} in batch")
    del rng


@pytest.mark.parametrize("flags", BATCH_FLAGS)
def test_batched_graphs_with_several_components(flags):
    """Each graph of the batch has several components (the frontier skips
    one sampled set per graph; the others must still be swept), including
    a large one next to small ones and a graph whose largest set is tiny."""
    rng = np.random.default_rng(17)
    graphs = []
    for i in range(24):
        pieces, base = [], 0
        for _ in range(int(rng.integers(2, 5))):
            m = int(rng.integers(3, 400 if i % 3 else 8))
            kind = int(rng.integers(0, 3))
            if kind == 0:
                pieces += [(base + a, base + b) for a, b in cycle(m)]
            elif kind == 1:
                pieces += [(base + a, base + b) for a, b in path(m)]
            else:
                pieces += [(base + a, base + (a + 1 + int(rng.integers(0, m - 1))) % m) for a in range(m)]
                pieces = [(a, b) for a, b in pieces if a != b]
            base += m + int(rng.integers(0, 5))  # isolated vertices between pieces
        graphs.append(gen.from_edges(base, pieces))
    u = gen.unite(graphs)
    note(f"batched multi-component graphs n={u.n} arcs={u.num_arcs} flags={flags:#x}")
    vb = torch.from_numpy(u.vbegin).to(DEV)
    off, adj = to_dev(u)
    r = solve_batched(vb, off, adj, flags=flags)
    torch.cuda.synchronize()
    lab, ap, nb = r.edge_label.cpu().numpy(), r.is_ap.cpu().numpy(), r.num_bcc.cpu().numpy()
    for i, g in enumerate(graphs):
        a0, a1 = u.offsets[u.vbegin[i]], u.offsets[u.vbegin[i + 1]]
        assert_parity(g, (lab[a0:a1], ap[u.vbegin[i] : u.vbegin[i + 1]], int(nb[i])), f"graph {i} in batch")


def test_validate_flag():
    g = gen.config("plain_small")
    note("validate ok")
    assert_parity(g, gpu_solve(g, flags=N.FLAG_VALIDATE), "validate")
    # asymmetric: drop one arc
    bad = gen.Csr(3, np.array([0, 1, 2, 2], np.int64), np.array([1, 0], np.int32))
    bad = gen.Csr(3, np.array([0, 2, 3, 3], np.int64), np.array([1, 2, 0], np.int32))
    note("validate asymmetric")
    off, adj = to_dev(bad)
    with pytest.raises(N.FastBccError) as ei:
        solve(off, adj, flags=N.FLAG_VALIDATE)
    assert ei.value.status == N.ERR_INVALID_GRAPH
    # out-of-range id
    bad = gen.Csr(2, np.array([0, 1, 2], np.int64), np.array([7, 0], np.int32))
    note("validate out-of-range")
    off, adj = to_dev(bad)
    with pytest.raises(N.FastBccError) as ei:
        solve(off, adj, flags=N.FLAG_VALIDATE)
    assert ei.value.status == N.ERR_INVALID_GRAPH


def test_validate_batched_graph_ranges():
    """Under validation a batch's graph ranges must run from 0 to n without
    decreasing, and no arc may leave its graph; a valid batch still solves."""
    graphs = [gen.from_edges(4, cycle(4)), gen.from_edges(3, path(3)), gen.from_edges(5, cycle(5))]
    u = gen.unite(graphs)
    off, adj = to_dev(u)
    note("validate batch: valid ranges")
    r = solve_batched(torch.from_numpy(u.vbegin).to(DEV), off, adj, flags=N.FLAG_VALIDATE)
    torch.cuda.synchronize()
    lab, nb = r.edge_label.cpu().numpy(), r.num_bcc.cpu().numpy()
    for i, g in enumerate(graphs):
        a0, a1 = u.offsets[u.vbegin[i]], u.offsets[u.vbegin[i + 1]]
        want, _, wnb, _, _ = oracle.ht_bcc(g.offsets, g.adj)
        assert np.array_equal(lab[a0:a1], want) and int(nb[i]) == wnb
    for bad, what in ((np.array([0, 4, 3, 12], np.int32), "decreasing"),
                      (np.array([0, 4, 7, 11], np.int32), "short of n"),
                      (np.array([1, 4, 7, 12], np.int32), "not from 0"),
                      (np.array([0, 3, 7, 12], np.int32), "an arc leaves its graph")):
        note(f"validate batch: {what}")
        with pytest.raises(N.FastBccError) as ei:
            solve_batched(torch.from_numpy(bad).to(DEV), off, adj, flags=N.FLAG_VALIDATE)
        assert ei.value.status == N.ERR_INVALID_GRAPH, what


def test_validate_loop_free_promise():
    """A self-loop is a valid input, but not under the loop-free flag: with
    validation on, breaking that promise is reported as an invalid graph."""
    loopy = gen.multigraph_csr(4, [(0, 1), (1, 2), (2, 0), (2, 3), (3, 3)])
    note("validate self-loop without the loop-free flag")
    assert_parity(loopy, gpu_solve(loopy, flags=N.FLAG_VALIDATE | N.FLAG_SORTED_ROWS), "self-loop")
    note("validate self-loop with the loop-free flag")
    off, adj = to_dev(loopy)
    with pytest.raises(N.FastBccError) as ei:
        solve(off, adj, flags=N.FLAG_VALIDATE | N.FLAG_SORTED_ROWS | N.FLAG_NO_SELF_LOOPS)
    assert ei.value.status == N.ERR_INVALID_GRAPH
    g = gen.config("rmat_small")
    note("validate loop-free rmat_small with the loop-free flag")
    flags = N.FLAG_VALIDATE | N.FLAG_SORTED_ROWS | N.FLAG_NO_SELF_LOOPS
    assert_parity(g, gpu_solve(g, flags=flags), "validated loop-free")


def test_traced_solve_same_result_and_times_kernels():
    from paper_2301_01356_amd import solve_traced

    g = gen.config("rmat_small")
    note("traced rmat_small")
    off, adj = to_dev(g)
    tr = N.Trace(max_launches=512)
    r = solve_traced(off, adj, tr)
    tr.collect()
    got = (r.edge_label.cpu().numpy(), r.is_ap.cpu().numpy(), int(r.num_bcc.item()))
    assert_parity(g, got, "traced")
    tot = tr.totals()
    for k in ("k_tag_sweep", "k_bcc_label", "k_lr_walk", "k_rmq_query", "k_cc_sweep", "k_lcc_sweep"):
        assert k in tot and tot[k][1] == 1 and tot[k][0] >= 0.0, k
    assert tr.dropped() == 0
    tr.close()


def vertex_sets_from_edge_labels(n, offsets, adj, lab):
    """BCC id -> vertex set, from canonical arc labels (unique: no tree involved)."""
    src = np.repeat(np.arange(n), np.diff(offsets))
    m = lab >= 0
    pairs = np.unique(np.stack([lab[m].astype(np.int64), src[m]], 1), axis=0)
    out = {}
    for c, v in pairs.tolist():
        out.setdefault(c, set()).add(v)
    return out


def check_bc_labeling(n, offsets, adj, oracle_lab, home, head, what):
    expect = vertex_sets_from_edge_labels(n, offsets, adj, oracle_lab)
    got = {}
    heads = {}
    for v in range(n):
        c = int(home[v])
        if c < 0:
            assert head[v] == -1
            continue
        got.setdefault(c, set()).add(v)
        h = int(head[v])
        assert heads.setdefault(c, h) == h, f"{what}: BCC {c} has two heads"
    for c, h in heads.items():
        assert h not in got[c], f"{what}: head of {c} is also a member"
        got[c].add(h)
    assert got == expect, f"{what}: BC-labeling does not reproduce the BCC vertex sets"


@pytest.mark.parametrize("name", ["plain_small", "grid_small", "rmat_small"])
def test_vertex_labels_reproduce_bcc_vertex_sets(name):
    from paper_2301_01356_amd import alloc_workspace, vertex_labels

    g = gen.config(name)
    note(f"vertex labels {name}")
    off, adj = to_dev(g)
    ws = alloc_workspace(g.n, g.num_arcs)
    solve(off, adj, workspace=ws)
    home, head = vertex_labels(ws, g.n, g.num_arcs)
    torch.cuda.synchronize()
    lab, ap, nb, _, _ = oracle.ht_bcc(g.offsets, g.adj)
    check_bc_labeling(g.n, g.offsets, g.adj, lab, home.cpu().numpy(), head.cpu().numpy(), name)
    # an articulation point is exactly a vertex that heads some BCC while also
    # belonging to another one (or heads two)
    h = head.cpu().numpy()
    hv = home.cpu().numpy()
    counts = np.bincount(h[h >= 0], minlength=g.n)
    heads_distinct = np.zeros(g.n, np.int64)
    for c in np.unique(hv[hv >= 0]):
        heads_distinct[h[np.flatnonzero(hv == c)[0]]] += 1
    is_ap = ((heads_distinct >= 1) & (hv >= 0)) | (heads_distinct >= 2)
    assert np.array_equal(is_ap.astype(np.uint8), ap)
    del counts


def test_vertex_labels_batched_are_graph_local():
    from paper_2301_01356_amd import alloc_workspace, vertex_labels

    graphs = [gen.mixed(71, i, 8, 1500, 4.0, 16.0) for i in range(12)]
    u = gen.unite(graphs)
    note("vertex labels batched")
    vb = torch.from_numpy(u.vbegin).to(DEV)
    off, adj = to_dev(u)
    ws = alloc_workspace(u.n, u.num_arcs, len(graphs))
    solve_batched(vb, off, adj, workspace=ws)
    home, head = vertex_labels(ws, u.n, u.num_arcs, vbegin=vb)
    torch.cuda.synchronize()
    home, head = home.cpu().numpy(), head.cpu().numpy()
    for i, g in enumerate(graphs):
        v0, v1 = u.vbegin[i], u.vbegin[i + 1]
        lab, _, _, _, _ = oracle.ht_bcc(g.offsets, g.adj)
        check_bc_labeling(g.n, g.offsets, g.adj, lab, home[v0:v1], head[v0:v1], f"graph {i}")


def hub_graph(seed=21):
    """Two hubs above every degree threshold of the solve (hub shards, long
    decomposition rows, long mirror searches): hub 0 with 12,000 pendant
    leaves and 1,500 triangles, hub 1 with 5,000 leaves, the hubs joined by
    three disjoint paths, a long pendant path, and random chords."""
    rng = np.random.default_rng(seed)
    edges = []
    nxt = 2
    for _ in range(12000):
        edges.append((0, nxt)); nxt += 1
    for _ in range(1500):
        a, b = nxt, nxt + 1; nxt += 2
        edges += [(0, a), (a, b), (b, 0)]
    for _ in range(5000):
        edges.append((1, nxt)); nxt += 1
    for _ in range(3):
        prev = 0
        for _ in range(50):
            edges.append((prev, nxt)); prev = nxt; nxt += 1
        edges.append((prev, 1))
    prev = 1
    for _ in range(3000):
        edges.append((prev, nxt)); prev = nxt; nxt += 1
    n = nxt
    for _ in range(400):
        u, v = int(rng.integers(2, n)), int(rng.integers(2, n))
        edges.append((u, v))
    return gen.from_edges(n, edges)


HUB_FLAGS = [
    0,
    N.FLAG_SORTED_ROWS,
    N.FLAG_SORTED_ROWS | N.tune_flags(sampled_tags=True),
    N.tune_flags(sampled_tags=True, cc_priority=True, tag_samples=2),
    N.tune_flags(ldd=1),
    N.FLAG_SORTED_ROWS | N.tune_flags(ldd=2, sample_rounds=0),
    N.FLAG_SORTED_ROWS | N.tune_flags(lcc_priority=True, free_first_round=True, lcc_rounds=0),
    N.FLAG_SORTED_ROWS | N.tune_flags(free_first_round=True, cc_priority=True, sampled_tags=True, tile_shift=5),
    N.FLAG_SORTED_ROWS | N.FLAG_NO_SELF_LOOPS | N.tune_flags(sampled_tags=True, free_first_round=True),
    N.FLAG_SORTED_ROWS | N.FLAG_NO_SELF_LOOPS | N.tune_flags(sampled_tags=True, tag_samples=1),
    N.FLAG_SORTED_ROWS | N.FLAG_NO_SELF_LOOPS,
]


@pytest.mark.parametrize("flags", HUB_FLAGS)
def test_hubs_above_every_degree_threshold(flags):
    g = hub_graph()
    note(f"hub graph n={g.n} arcs={g.num_arcs} max degree={int(np.diff(g.offsets).max())} flags={flags:#x}")
    assert_parity(g, gpu_solve(g, flags=flags), f"hub graph {flags:#x}")


@pytest.mark.parametrize("flags", HUB_FLAGS[:3] + HUB_FLAGS[-2:])
def test_hub_graphs_batched(flags):
    graphs = [hub_graph(21), gen.from_edges(5, cycle(5)), hub_graph(22)]
    u = gen.unite(graphs)
    note(f"batched hub graphs n={u.n} arcs={u.num_arcs} flags={flags:#x}")
    vb = torch.from_numpy(u.vbegin).to(DEV)
    off = torch.from_numpy(u.offsets32()).to(DEV)
    adj = torch.from_numpy(u.adj).to(DEV)
    r = solve_batched(vb, off, adj, flags=flags)
    torch.cuda.synchronize()
    lab, ap, nb = r.edge_label.cpu().numpy(), r.is_ap.cpu().numpy(), r.num_bcc.cpu().numpy()
    for i, gi in enumerate(graphs):
        v0, v1 = int(u.vbegin[i]), int(u.vbegin[i + 1])
        a0, a1 = int(u.offsets[v0]), int(u.offsets[v1])
        assert_parity(gi, (lab[a0:a1], ap[v0:v1], int(nb[i])), f"batched hub graph {i}")


@pytest.mark.parametrize("flags", [0, N.tune_flags(xcd_order=True), N.tune_flags(xcd_order=True, graph_cc=True)])
@pytest.mark.parametrize("sizes", [(200, 56, 256), (256, 256), (100, 156, 300, 212), (512,), (30, 226),
                                   (256,) * 9 + (100,)])
def test_batched_counts_when_the_batch_ends_on_a_block_boundary(sizes, flags):
    """Per-graph BCC counts read the scanned per-block counts up to the end
    of the last graph; when the vertex total is a multiple of the block size
    (256) that is the scan's total slot.  The workspace starts full of
    garbage so that a slot the solve did not write cannot pass by luck; the
    same with XCD-ordered launches and with the per-graph passes."""
    rng = np.random.default_rng(sum(sizes))
    graphs = []
    for n in sizes:
        edges = [(i, i + 1) for i in range(n - 1)]  # a path: n - 1 BCCs
        edges += [(int(rng.integers(0, n)), int(rng.integers(0, n))) for _ in range(n // 3)]
        graphs.append(gen.from_edges(n, [(a, b) for a, b in edges if a != b]))
    u = gen.unite(graphs)
    assert u.n % 256 == 0 or len(sizes) == 2 or sizes[-1] == 100
    vb = torch.from_numpy(u.vbegin).to(DEV)
    off, adj = to_dev(u)
    ws = alloc_workspace(u.n, u.num_arcs, len(graphs), DEV)
    for fill in (0x7F, 0x00, 0xFF):
        ws.fill_(fill)
        note(f"batch ending on a block boundary: sizes {sizes}, n={u.n}, workspace fill {fill:#x}, flags {flags:#x}")
        r = solve_batched(vb, off, adj, workspace=ws, flags=flags)
        lab, ap, nb = r.edge_label.cpu().numpy(), r.is_ap.cpu().numpy(), r.num_bcc.cpu().numpy()
        for i, g in enumerate(graphs):
            a0, a1 = u.offsets[u.vbegin[i]], u.offsets[u.vbegin[i + 1]]
            assert_parity(g, (lab[a0:a1], ap[u.vbegin[i] : u.vbegin[i + 1]], int(nb[i])), f"graph {i} fill {fill:#x}")


def test_priority_last_cc_labels_stable_over_repeated_solves():
    """Last-CC hooking by priority relabels every set to its smallest member
    and the read-out reads lab[v] as the label, so every entry must sit on its
    set's root after the last compression.  Concurrent path halving could
    leave an entry on a stale ancestor, which split a BCC in about one solve
    in a thousand on this tree-like graph; the flattening pass that reads only
    rules that out.  2000 solves, each compared with the oracle on the device."""
    from paper_2301_01356_amd.serve import serving_flags

    g = gen.mixed(5, 2, 1 << 10, 1 << 22, 4.0, 32.0)
    lab, ap, nb, _, _ = oracle.ht_bcc(g.offsets, g.adj)
    off, adj = to_dev(g)
    rl = torch.from_numpy(lab).to(DEV)
    ra = torch.from_numpy(ap).to(DEV)
    ws = alloc_workspace(g.n, g.num_arcs, 1, DEV)
    flags = serving_flags()
    note(f"2000 priority Last-CC solves n={g.n} arcs={g.num_arcs} flags={flags:#x}")
    bad = torch.zeros((), dtype=torch.int64, device=DEV)
    for _ in range(2000):
        r = solve(off, adj, workspace=ws, flags=flags)
        bad += (r.edge_label != rl).any() | (r.is_ap != ra).any() | (r.num_bcc[0] != nb)
    assert int(bad.item()) == 0
    assert read_device_status(ws) == 0


@pytest.mark.parametrize("flags", [N.tune_flags(graph_cc=True),
                                   N.FLAG_SORTED_ROWS | N.FLAG_NO_SELF_LOOPS | N.tune_flags(graph_cc=True)])
def test_batched_per_graph_first_cc_sizes(flags):
    """Per-graph First-CC across its size boundary: graphs of 2^16 - 1 and 2^16
    vertices keep their parents in LDS, one of 2^16 + 1 and a larger one run
    on the device-memory union-find; with empty, edgeless and tiny graphs
    and a disconnected one around them."""
    lim = 1 << 16
    empty = gen.Csr(0, np.zeros(1, np.int64), np.zeros(0, np.int32))
    edgeless = gen.Csr(5, np.zeros(6, np.int64), np.zeros(0, np.int32))
    two = gen.unite([gen.family("knn", 3000, 5, seed=7), gen.family("random", 2000, 3.0, seed=8)])
    two = gen.Csr(two.n, two.offsets, two.adj)
    graphs = [gen.family("lattice", lim, 0.75, seed=1), empty, gen.family("random", lim - 1, 6.0, seed=2),
              edgeless, gen.family("tree_back", lim + 1, 0.2, seed=3), gen.from_edges(3, cycle(3)), two,
              gen.family("knn", 90000, 5, seed=4), empty, gen.family("lattice", 700, 0.8, seed=5)]
    u = gen.unite(graphs)
    note(f"per-graph First-CC: {len(graphs)} graphs n={u.n} arcs={u.num_arcs} flags={flags:#x}")
    vb = torch.from_numpy(u.vbegin).to(DEV)
    off, adj = to_dev(u)
    r = solve_batched(vb, off, adj, flags=flags)
    torch.cuda.synchronize()
    lab, ap, nb = r.edge_label.cpu().numpy(), r.is_ap.cpu().numpy(), r.num_bcc.cpu().numpy()
    for i, g in enumerate(graphs):
        a0, a1 = u.offsets[u.vbegin[i]], u.offsets[u.vbegin[i + 1]]
        assert_parity(g, (lab[a0:a1], ap[u.vbegin[i] : u.vbegin[i + 1]], int(nb[i])), f"graph {i} (n={g.n})")


@pytest.mark.parametrize("flags", [N.tune_flags(graph_cc=True),
                                   N.FLAG_SORTED_ROWS | N.FLAG_NO_SELF_LOOPS | N.tune_flags(graph_cc=True)])
def test_batched_per_graph_more_graphs_than_vertices(flags):
    """The per-graph passes take the graphs largest first when the batch has
    at most as many graphs as vertices, else in index order: a batch of
    mostly empty graphs (more graphs than vertices) around a few small ones."""
    empty = gen.Csr(0, np.zeros(1, np.int64), np.zeros(0, np.int32))
    small = [gen.from_edges(4, cycle(4)), gen.from_edges(3, path(3)), gen.family("random", 9, 2.0, seed=3)]
    graphs = [empty] * 7 + [small[0]] + [empty] * 11 + [small[1], small[2]] + [empty] * 5
    u = gen.unite(graphs)
    assert len(graphs) > u.n
    note(f"per-graph passes, {len(graphs)} graphs n={u.n} arcs={u.num_arcs} flags={flags:#x}")
    vb = torch.from_numpy(u.vbegin).to(DEV)
    off, adj = to_dev(u)
    r = solve_batched(vb, off, adj, flags=flags)
    torch.cuda.synchronize()
    lab, ap, nb = r.edge_label.cpu().numpy(), r.is_ap.cpu().numpy(), r.num_bcc.cpu().numpy()
    for i, g in enumerate(graphs):
        a0, a1 = u.offsets[u.vbegin[i]], u.offsets[u.vbegin[i + 1]]
        assert_parity(g, (lab[a0:a1], ap[u.vbegin[i] : u.vbegin[i + 1]], int(nb[i])), f"graph {i} (n={g.n})")


@pytest.mark.parametrize("flags", [N.tune_flags(graph_cc=True), N.tune_flags(graph_cc=True, xcd_order=True)])
def test_batched_per_graph_long_rows_outside_the_largest_set(flags):
    """The per-graph sweeps spread the rows outside each graph's largest set
    over a wave's lanes: hubs of thousands of arcs outside it (a star beside a
    larger lattice, a star whose hub has the largest id, a star inside a graph
    above the LDS size), repeated edges and self-loops (general contract)."""
    rng = np.random.default_rng(23)

    def star_beside(base_n, leaves, hub_last):
        lat = gen.family("lattice", base_n, 0.9, seed=int(rng.integers(1 << 30)))
        ed = []
        for v in range(lat.n):
            for a in range(int(lat.offsets[v]), int(lat.offsets[v + 1])):
                if v < int(lat.adj[a]):
                    ed.append((v, int(lat.adj[a])))
        hub = lat.n + leaves if hub_last else lat.n
        first_leaf = lat.n if hub_last else lat.n + 1
        ed += [(hub, first_leaf + i) for i in range(leaves)]
        ed += [(first_leaf + i, first_leaf + i + 1) for i in range(0, leaves - 1, 7)]  # a few leaf-leaf chords
        return gen.multigraph_csr(lat.n + leaves + 1, ed)

    loopy = gen.multigraph_csr(6, [(0, 1), (0, 1), (1, 2), (2, 0), (2, 2), (3, 4), (4, 5), (5, 3), (5, 5), (2, 3)])
    graphs = [star_beside(4000, 3000, False), loopy, star_beside(2500, 5000, True),
              star_beside(70000, 4000, False), gen.from_edges(3, cycle(3))]
    u = gen.unite(graphs)
    note(f"per-graph long rows: {len(graphs)} graphs n={u.n} arcs={u.num_arcs} flags={flags:#x}")
    vb = torch.from_numpy(u.vbegin).to(DEV)
    off, adj = to_dev(u)
    r = solve_batched(vb, off, adj, flags=flags)
    torch.cuda.synchronize()
    lab, ap, nb = r.edge_label.cpu().numpy(), r.is_ap.cpu().numpy(), r.num_bcc.cpu().numpy()
    for i, g in enumerate(graphs):
        a0, a1 = u.offsets[u.vbegin[i]], u.offsets[u.vbegin[i + 1]]
        assert_parity(g, (lab[a0:a1], ap[u.vbegin[i] : u.vbegin[i + 1]], int(nb[i])), f"graph {i} (n={g.n})")
