"""The padded union that the batched solver feeds the GPU is always a valid
symmetric CSR (ids in range, offsets monotone, rows sorted, every arc count
covered), and its BCC structure is exactly the union of the graphs' own plus
the padding graph's one 2-cycle (CPU oracle)."""
import numpy as np
import pytest

import oracle
from paper_2301_01356_amd import gen
from paper_2301_01356_amd.batch import pack
from paper_2301_01356_amd.serve import check_request


def as_csr(vb, off, adj):
    return gen.Csr(off.shape[0] - 1, off.astype(np.int64), adj)


@pytest.mark.parametrize("count", [0, 1, 7, 30])
def test_pack_is_valid_and_preserves_bccs(count):
    graphs = [gen.mixed(61, i, 4, 900, 4.0, 16.0) for i in range(count)]
    cap_v = sum(g.n for g in graphs) + 37
    cap_a = sum(g.num_arcs for g in graphs) + 101
    vb, off, adj, spans = pack(graphs, cap_v, cap_a, 40)
    u = as_csr(vb, off, adj)
    assert check_request(u) == ""
    assert vb[0] == 0 and vb[-1] == cap_v and np.all(np.diff(vb) >= 0)
    assert off[-1] == cap_a and np.all(np.diff(off.astype(np.int64)) >= 0)
    assert adj.min() >= 0 and adj.max() < cap_v
    lab, ap, nb, _, _ = oracle.ht_bcc(u.offsets, u.adj)
    total = 0
    for g, (v0, v1, a0, a1) in zip(graphs, spans):
        glab, gap, gnb, _, _ = oracle.ht_bcc(g.offsets, g.adj)
        sub = lab[a0:a1]
        np.testing.assert_array_equal(np.where(sub >= 0, sub - a0, -1), glab)
        np.testing.assert_array_equal(ap[v0:v1], gap)
        total += gnb
    # the padding: parallel copies of one edge (one BCC, labelled by its first
    # arc), a self-loop for an odd leftover arc, no articulation point
    a_used = spans[-1][3] if spans else 0
    left = cap_a - a_used
    assert nb == total + (1 if left >= 2 else 0)
    assert ap[spans[-1][1] if spans else 0 :].sum() == 0
    assert np.all(lab[a_used : cap_a - (left & 1)] == a_used)
    if left & 1:
        assert lab[cap_a - 1] == -1
    for v in range(u.n):
        row = u.adj[u.offsets[v] : u.offsets[v + 1]]
        assert np.all(row[1:] >= row[:-1]), "padded rows must stay sorted"


@pytest.mark.parametrize("left", [0, 1, 2, 9])
def test_pack_padding_is_loop_free_for_even_leftovers(left):
    g = gen.from_edges(4, [(0, 1), (1, 2), (2, 3), (3, 0)])
    vb, off, adj, spans = pack([g], 4 + 2, g.num_arcs + left, 2)
    u = as_csr(vb, off, adj)
    src = np.repeat(np.arange(u.n), np.diff(u.offsets))
    assert int((src == u.adj).sum()) == (left & 1)


def test_pack_rejects_overflow():
    g = gen.from_edges(10, [(i, i + 1) for i in range(9)])
    with pytest.raises(ValueError):
        pack([g], 11, 100, 4)  # needs two spare vertices for leftover arcs
    pack([g], 12, 100, 4)
    pack([g], 11, 18, 4)  # no leftover arcs: one spare vertex
    with pytest.raises(ValueError):
        pack([g] * 5, 1000, 1000, 4)


def test_greedy_packs_bounds_every_pack():
    from paper_2301_01356_amd import _native as N
    from paper_2301_01356_amd.api import greedy_packs

    rng = np.random.default_rng(5)
    sizes = list(rng.integers(0, 900, size=500)) + [3000, 0, 0, 5] + [0] * 4000
    for cap in (256, 1024, 3072):
        p = greedy_packs(sizes, cap)
        assert p[0] == 0 and p[-1] == len(sizes) and all(a < b for a, b in zip(p, p[1:]))
        for a, b in zip(p, p[1:]):
            tot = sum(sizes[a:b])
            assert b - a <= N.SMALL_MAX_VERTICES
            assert tot <= cap or b - a == 1, "only a single graph may exceed the capacity"
            if b < len(sizes) and b - a < N.SMALL_MAX_VERTICES:
                assert tot + sizes[b] > cap, "greedy: the next graph did not fit"
    assert greedy_packs([], 10) == [0]


def test_split_capacities():
    from paper_2301_01356_amd import gen
    from paper_2301_01356_amd.batch import SplitBatchedSolver

    graphs = [gen.mixed(7, i, 16, 6000, 4.0, 8.0) for i in range(40)]
    (sv, sa, sg), (bv, ba, bg) = SplitBatchedSolver.capacities(graphs, 3072)
    small = [g for g in graphs if g.n <= 3072]
    big = [g for g in graphs if g.n > 3072]
    assert sg == max(len(small), 1) and bg == max(len(big), 1)
    assert sv == sum(g.n for g in small) + 2 and bv == sum(g.n for g in big) + 2
    assert sa == max(sum(g.num_arcs for g in small), 1) and ba == max(sum(g.num_arcs for g in big), 1)
