"""The Tarjan-Vishkin test solver (explicit skeleton, breadth-first tree)
agrees with the Hopcroft-Tarjan oracle and with brute force."""
import numpy as np
import pytest

import oracle
from oracle.tv_bcc import tv_bcc
from paper_2301_01356_amd import gen
from tests import bruteforce as bf


def test_tv_matches_bruteforce_on_random_multigraphs():
    rng = np.random.default_rng(21)
    for _ in range(300):
        n = int(rng.integers(1, 9))
        m = int(rng.integers(0, 14))
        edges = [(int(rng.integers(0, n)), int(rng.integers(0, n))) for _ in range(m)]
        edges += edges[: int(rng.integers(0, 3))]
        g = gen.multigraph_csr(n, edges)
        lab, ap, nb = tv_bcc(g.offsets, g.adj)
        elab, eap, enb = bf.expected_from_csr(n, g.offsets, g.adj)
        assert nb == enb, edges
        np.testing.assert_array_equal(lab, elab, err_msg=str(edges))
        np.testing.assert_array_equal(ap, eap, err_msg=str(edges))


@pytest.mark.parametrize("name", ["plain_small", "grid_small", "rmat_small", "batch_small"])
def test_tv_matches_hopcroft_tarjan(name):
    g = gen.config(name)
    lab, ap, nb, _, _ = oracle.ht_bcc(g.offsets, g.adj)
    tlab, tap, tnb, size = tv_bcc(g.offsets, g.adj, return_skeleton_size=True)
    assert tnb == nb
    np.testing.assert_array_equal(tlab, lab)
    np.testing.assert_array_equal(tap, ap)
    # the skeleton has one vertex per edge and O(m) edges (paper's space argument)
    assert size["skeleton_vertices"] == g.num_arcs // 2
    assert size["skeleton_edges"] <= 2 * size["skeleton_vertices"]
