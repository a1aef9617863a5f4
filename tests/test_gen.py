"""The seeded input generators (CPU): every graph is a valid symmetric CSR with
sorted, merged, loop-free rows; output depends on the seed alone, not on the
number of threads; the plain workload has the sizes its recipe states."""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2301_01356_amd import gen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SMALL = ["plain_small", "grid_small", "rmat_small", "batch_small"]


def check_csr(g):
    off = np.asarray(g.offsets, np.int64)
    adj = np.asarray(g.adj, np.int64)
    assert off.shape == (g.n + 1,) and off[0] == 0 and off[-1] == adj.size
    assert np.all(np.diff(off) >= 0)
    if adj.size == 0:
        return
    assert adj.min() >= 0 and adj.max() < g.n
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(off))
    assert not np.any(src == adj), "self-loop"
    # strictly increasing inside every row: sorted and merged
    inner = np.ones(adj.size, bool)
    inner[off[:-1][np.diff(off) > 0]] = False
    assert np.all(np.diff(adj)[inner[1:]] > 0)
    # symmetric: the arc set equals its reverse
    fwd = np.sort(src * g.n + adj)
    rev = np.sort(adj * g.n + src)
    assert np.array_equal(fwd, rev)


@pytest.mark.parametrize("name", SMALL)
def test_small_configs_are_valid_symmetric_csr(name):
    check_csr(gen.config(name))


def test_united_batch_is_valid_and_graphs_stay_apart():
    graphs = [gen.mixed(7, i, 8, 500, 4.0, 16.0) for i in range(12)]
    u = gen.unite(graphs)
    check_csr(u)
    vb = np.asarray(u.vbegin, np.int64)
    for i in range(len(graphs)):
        a0, a1 = u.offsets[vb[i]], u.offsets[vb[i + 1]]
        seg = np.asarray(u.adj[a0:a1], np.int64)
        assert seg.size == 0 or (seg.min() >= vb[i] and seg.max() < vb[i + 1])


def test_same_seed_same_graph_other_seed_other_graph():
    a, b, c = gen.rmat(seed=13, scale=12), gen.rmat(seed=13, scale=12), gen.rmat(seed=14, scale=12)
    assert np.array_equal(a.offsets, b.offsets) and np.array_equal(a.adj, b.adj)
    assert not (a.adj.size == c.adj.size and np.array_equal(a.adj, c.adj))


def _digest_in_subprocess(threads):
    code = ("import hashlib, sys; sys.path.insert(0, %r)\n"
            "from paper_2301_01356_amd import gen\n"
            "h = hashlib.sha256()\n"
            "for name in ('rmat_small', 'batch_small', 'grid_small'):\n"
            "    g = gen.config(name); h.update(g.offsets.tobytes()); h.update(g.adj.tobytes())\n"
            "print(h.hexdigest())\n") % ROOT
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr
    return r.stdout.strip()


def test_output_does_not_depend_on_thread_count():
    assert _digest_in_subprocess(1) == _digest_in_subprocess(8)


def test_plain_workload_sizes_match_its_recipe():
    g = gen.config("plain")
    assert (g.n, g.num_arcs) == (202_076, 1_190_678)
