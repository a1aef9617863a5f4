"""The padded union that the batched solver feeds the GPU is always a valid
symmetric CSR (ids in range, offsets monotone, every arc count covered), and
its BCC structure is exactly the union of the graphs' own (CPU oracle)."""
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
    # the padding (self-loops on one vertex) adds no BCC and no articulation point
    assert nb == total
    assert ap[spans[-1][1] if spans else 0 :].sum() == 0
    assert np.all(lab[spans[-1][3] if spans else 0 :] == -1)


def test_pack_rejects_overflow():
    g = gen.from_edges(10, [(i, i + 1) for i in range(9)])
    with pytest.raises(ValueError):
        pack([g], 10, 100, 4)  # needs one spare vertex for padding
    with pytest.raises(ValueError):
        pack([g] * 5, 1000, 1000, 4)
