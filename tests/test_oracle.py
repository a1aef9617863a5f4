"""Pins for the CPU oracle (Hopcroft-Tarjan), all on the CPU.

The oracle is checked against things other than itself:
  * brute force from the definitions (every simple graph on 6 labelled
    vertices; random multigraphs with loops on up to 10 vertices),
  * closed forms (cycles, paths, trees, stars, complete graphs, grids, tori,
    two cycles sharing a vertex, barbells),
  * the paper's Table 1 synthetic rows (chains; full and p=0.6 tori),
  * planted structures in the benchmark generators,
  * block-cut-tree identities that any correct BCC partition satisfies.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2301_01356_amd import gen
from tests import bruteforce as bf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_table1_synthetic.json")


def run(g):
    lab, ap, nb, _, _ = oracle.ht_bcc(g.offsets, g.adj)
    return lab, ap, nb


# ------------------------------------------------------------ brute force
def test_exhaustive_all_graphs_on_6_vertices():
    n = 6
    pairs, cmasks = bf.complete_graph_cycles(n)
    P = len(pairs)
    for g in range(1 << P):
        bits = [i for i in range(P) if (g >> i) & 1]
        local = {b: k for k, b in enumerate(bits)}
        contained = cmasks[(cmasks & ~g) == 0]
        cycles = [frozenset(local[i] for i in range(P) if (int(m) >> i) & 1) for m in contained]
        edges = [pairs[i] for i in bits]
        csr = gen.from_edges(n, edges) if edges else gen.Csr(n, np.zeros(n + 1, np.int64), np.zeros(0, np.int32))
        lab, ap, nb = run(csr)
        elab, eap, enb = bf.expected_from_csr(n, csr.offsets, csr.adj, cycles=cycles, pairs=edges)
        assert nb == enb, (g, edges)
        np.testing.assert_array_equal(lab, elab, err_msg=str(edges))
        np.testing.assert_array_equal(ap, eap, err_msg=str(edges))


@pytest.mark.parametrize("seed", range(4))
def test_random_multigraphs_with_loops_vs_bruteforce(seed):
    rng = np.random.default_rng(1000 + seed)
    for _ in range(400):
        n = int(rng.integers(2, 11))
        m = int(rng.integers(0, 15))
        edges = [(int(rng.integers(0, n)), int(rng.integers(0, n))) for _ in range(m)]
        # a few deliberate parallel copies
        for _ in range(int(rng.integers(0, 3))):
            if edges:
                edges.append(edges[int(rng.integers(0, len(edges)))])
        csr = gen.multigraph_csr(n, edges)
        if rng.random() < 0.5:
            # rows need not be sorted: shuffle inside every row
            adj = csr.adj.copy()
            for v in range(n):
                s, e = csr.offsets[v], csr.offsets[v + 1]
                adj[s:e] = rng.permutation(adj[s:e])
            csr = gen.Csr(n, csr.offsets, adj)
        lab, ap, nb = run(csr)
        elab, eap, enb = bf.expected_from_csr(n, csr.offsets, csr.adj)
        assert nb == enb, edges
        np.testing.assert_array_equal(lab, elab, err_msg=str(edges))
        np.testing.assert_array_equal(ap, eap, err_msg=str(edges))


# ------------------------------------------------------------ closed forms
def cycle(n):
    return [(i, (i + 1) % n) for i in range(n)]


def path(n):
    return [(i, i + 1) for i in range(n - 1)]


def counts(n, edges):
    g = gen.from_edges(n, edges)
    lab, ap, nb = run(g)
    return nb, int(ap.sum()), g, lab, ap


@pytest.mark.parametrize("n", [3, 4, 17, 1000])
def test_cycle_is_one_bcc(n):
    nb, nap, *_ = counts(n, cycle(n))
    assert (nb, nap) == (1, 0)


@pytest.mark.parametrize("n", [2, 3, 10, 5000])
def test_path_has_n_minus_1_bccs(n):
    nb, nap, *_ = counts(n, path(n))
    assert (nb, nap) == (n - 1, n - 2)


def test_random_tree_every_edge_is_a_bcc():
    rng = np.random.default_rng(5)
    n = 3000
    edges = [(int(rng.integers(0, i)), i) for i in range(1, n)]
    nb, nap, g, lab, ap = counts(n, edges)
    assert nb == n - 1
    deg = np.diff(g.offsets)
    np.testing.assert_array_equal(ap, (deg >= 2).astype(np.uint8))


@pytest.mark.parametrize("k", [1, 2, 50])
def test_star(k):
    nb, nap, *_ = counts(k + 1, [(0, i) for i in range(1, k + 1)])
    assert nb == k and nap == (1 if k >= 2 else 0)


@pytest.mark.parametrize("n", [3, 4, 9])
def test_complete_graph_one_bcc(n):
    edges = [(i, j) for i in range(n) for j in range(i + 1, n)]
    assert counts(n, edges)[:2] == (1, 0)


@pytest.mark.parametrize("rows,cols,wrap", [(2, 2, False), (7, 13, False), (40, 40, False), (5, 9, True), (30, 50, True)])
def test_full_grid_and_torus_one_bcc(rows, cols, wrap):
    g = gen.grid(seed=1, rows=rows, cols=cols, p=1.0, path_len=0, wrap=wrap)
    lab, ap, nb = run(g)
    assert nb == 1 and ap.sum() == 0


def test_two_cycles_sharing_a_vertex():
    a = cycle(5)
    b = [(0, 5), (5, 6), (6, 7), (7, 0)]
    nb, nap, g, lab, ap = counts(8, a + b)
    assert (nb, nap) == (2, 1) and ap[0] == 1


@pytest.mark.parametrize("k,L", [(3, 1), (4, 3), (6, 10)])
def test_barbell(k, L):
    # two K_k joined by a path of L edges: L + 2 BCCs, L + 1 articulation points
    e = [(i, j) for i in range(k) for j in range(i + 1, k)]
    e += [(k + i, k + j) for i in range(k) for j in range(i + 1, k)]
    chain = [k - 1] + [2 * k + t for t in range(L - 1)] + [k]
    e += [(chain[t], chain[t + 1]) for t in range(L)]
    n = 2 * k + L - 1
    assert counts(n, e)[:2] == (L + 2, L + 1)


def test_isolated_vertices_and_empty_graph():
    g = gen.Csr(5, np.zeros(6, np.int64), np.zeros(0, np.int32))
    lab, ap, nb = run(g)
    assert nb == 0 and ap.sum() == 0 and lab.size == 0
    nb, nap, *_ = counts(6, [(1, 2)])
    assert (nb, nap) == (1, 0)


def test_self_loops_and_parallel_edges():
    g = gen.multigraph_csr(3, [(0, 0), (0, 1), (0, 1), (1, 2), (2, 2)])
    lab, ap, nb = run(g)
    # arcs: row0: 0->0, 0->1, 0->1 ; row1: 1->0, 1->0, 1->2 ; row2: 2->1, 2->2
    assert nb == 2
    np.testing.assert_array_equal(lab, [-1, 1, 1, 1, 1, 5, 5, -1])
    np.testing.assert_array_equal(ap, [0, 1, 0])


def test_rejects_asymmetric_csr():
    g = gen.Csr(2, np.array([0, 1, 1], np.int64), np.array([1], np.int32))
    with pytest.raises(oracle.OracleError):
        run(g)


# ------------------------------------------------------------ paper Table 1
def test_table1_chain_rows_scaled():
    gold = json.load(open(GOLDEN))["rows"]
    # Chn7/Chn8: a chain of n vertices has n - 1 BCCs; checked at 10^5 and 10^6
    assert gold["Chn7"]["num_bcc"] == gold["Chn7"]["n"] - 1
    for n in (10**5, 10**6):
        g = gen.from_edges(n, path(n))
        lab, ap, nb = run(g)
        assert nb == n - 1 and int(ap.sum()) == n - 2


def test_table1_full_tori_one_bcc():
    gold = json.load(open(GOLDEN))["rows"]
    assert gold["SQR"]["num_bcc"] == 1 and gold["REC"]["num_bcc"] == 1
    for r, c in ((300, 300), (30, 3000)):
        g = gen.grid(seed=3, rows=r, cols=c, p=1.0, path_len=0, wrap=True)
        assert run(g)[2] == 1


def largest_bcc_vertex_fraction(g, lab):
    n = g.n
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.offsets))
    m = lab >= 0
    pairs = np.unique(lab[m].astype(np.int64) * n + src[m])
    _, cnt = np.unique(pairs // n, return_counts=True)
    return cnt.max() / n


@pytest.mark.parametrize("row,rows,cols", [("SQR'", 2000, 2000), ("REC'", 400, 10000)])
def test_table1_sampled_tori_statistics(row, rows, cols):
    gold = json.load(open(GOLDEN))["rows"][row]
    g = gen.grid(seed=21, rows=rows, cols=cols, p=gold["p"], path_len=0, wrap=True)
    lab, ap, nb = run(g)
    per_vertex = gold["num_bcc"] / gold["n"]
    assert abs(nb / g.n - per_vertex) / per_vertex < 0.01
    assert abs(100.0 * largest_bcc_vertex_fraction(g, lab) - gold["largest_bcc_pct"]) < 1.0


# ------------------------------------------------------------ planted structure
def test_plain_config_planted_counts():
    kw = dict(seed=11, n_base=1 << 12, m_base=1 << 14, n_pendant=64, n_cycles=8, cmin=10, cmax=60)
    g = gen.plain(**kw)
    base = gen.plain(**{**kw, "n_pendant": 0, "n_cycles": 0})
    n_base, pend_total, n_cycles = g.meta.tolist()
    # a pendant tree of s vertices hung by one edge gives s bridges; a cycle
    # hung by one bridge gives 2 BCCs; the base graph keeps its own BCCs
    assert run(g)[2] == run(base)[2] + pend_total + 2 * n_cycles


def test_grid_config_planted_path_counts():
    kw = dict(seed=12, rows=128, cols=96, path_len=5000, chord_block=100)
    g = gen.grid(**kw)
    lattice = gen.grid(**{**kw, "path_len": 0})
    rows, cols, plen, corner = g.meta.tolist()
    base = rows * cols
    src = np.repeat(np.arange(g.n), np.diff(g.offsets))
    sel = (src >= base) & (g.adj > src) & (g.adj >= base) & (g.adj - src >= 2)
    chords = np.stack([src[sel] - base, g.adj[sel] - base], 1)
    assert len(chords) == (plen + 99) // 100
    # path edges + the attaching edge are bridges except those a chord closes
    expected = run(lattice)[2] + plen - int(np.sum(chords[:, 1] - chords[:, 0] - 1))
    assert run(g)[2] == expected


# ------------------------------------------------------------ invariants
def check_partition_invariants(g, lab, ap, nb):
    n = g.n
    off = g.offsets
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(off))
    adj = g.adj.astype(np.int64)
    # both arcs of an edge share the label (rows sorted, simple graph)
    for a in np.random.default_rng(0).choice(len(adj), size=min(2000, len(adj)), replace=False):
        u, v = src[a], adj[a]
        b = off[v] + np.searchsorted(g.adj[off[v] : off[v + 1]], u)
        assert lab[b] == lab[a]
    # every label is the smallest arc of its own class
    m = lab >= 0
    assert np.all(lab[m] <= np.nonzero(m)[0])
    assert np.all(lab[lab[m]] == lab[m])
    labels = np.unique(lab[m])
    assert len(labels) == nb
    # vertex-BCC incidences
    inc = np.unique(lab[m].astype(np.int64) * n + src[m])
    inc_v = inc % n
    inc_l = inc // n
    per_vertex = np.bincount(inc_v, minlength=n)
    # articulation point iff the vertex lies in two or more BCCs
    np.testing.assert_array_equal(ap, (per_vertex >= 2).astype(np.uint8))
    # block-cut forest: per connected component with an edge,
    # sum_C (|V(C)| - 1) = |CC| - 1 and sum_v (bcc(v) - 1) = #BCC - 1
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components

    A = sp.csr_matrix((np.ones(len(adj)), adj, off), shape=(n, n))
    ncc, cc = connected_components(A, directed=False)
    sizes = np.bincount(inc_l, minlength=0)
    size_of = sizes[labels]
    cc_of_label = cc[src[labels]]
    lhs = np.bincount(cc_of_label, weights=size_of - 1, minlength=ncc)
    ccsize = np.bincount(cc, minlength=ncc)
    has_edge = np.bincount(cc_of_label, minlength=ncc) > 0
    np.testing.assert_array_equal(lhs[has_edge], ccsize[has_edge] - 1)
    bccs_per_cc = np.bincount(cc_of_label, minlength=ncc)
    inv = np.bincount(cc[inc_v], weights=np.ones(len(inc_v)), minlength=ncc)  # sum_v bcc(v)
    nonisolated = np.bincount(cc[np.unique(inc_v)], minlength=ncc)
    np.testing.assert_array_equal((inv - nonisolated)[has_edge], bccs_per_cc[has_edge] - 1)
    # two BCCs share at most one vertex
    order = np.argsort(inc_v, kind="stable")
    v_sorted, l_sorted = inc_v[order], inc_l[order]
    pair_keys = []
    starts = np.flatnonzero(np.r_[True, v_sorted[1:] != v_sorted[:-1]])
    ends = np.r_[starts[1:], len(v_sorted)]
    for s, e in zip(starts, ends):
        if e - s >= 2:
            ls = l_sorted[s:e]
            for i in range(len(ls)):
                for j in range(i + 1, len(ls)):
                    pair_keys.append(min(ls[i], ls[j]) * (1 << 31) + max(ls[i], ls[j]))
    if pair_keys:
        _, c = np.unique(np.array(pair_keys, np.int64), return_counts=True)
        assert c.max() == 1


@pytest.mark.parametrize("name", ["plain_small", "grid_small", "rmat_small", "batch_small"])
def test_oracle_output_invariants(name):
    g = gen.config(name)
    check_partition_invariants(g, *run(g))
