"""Serving scheduler on the CPU: simulated clock, simulated slots and the
CPU oracle as the solver (the scheduler is the code under test here)."""
import numpy as np
import pytest

import oracle
from paper_2301_01356_amd import gen
from paper_2301_01356_amd.serve import Request, Server, SimClock, SimSlot, latency_summary, poisson_arrivals, request_bytes


def oracle_solve(g):
    lab, ap, nb, _, _ = oracle.ht_bcc(g.offsets, g.adj)
    return lab, ap, nb


def make_requests(count, seed=7, qps=2000.0, nmax=3000):
    arr = poisson_arrivals(count, qps, seed)
    return [Request(i, gen.mixed(seed, i, 16, nmax, 4.0, 16.0), float(arr[i])) for i in range(count)]


def server(slots=2, cap_v=20000, cap_a=200000, cap_g=64, budget=1 << 40, cost=None):
    clk = SimClock()
    ss = [SimSlot(clk, oracle_solve, cap_v, cap_a, cap_g, cost) for _ in range(slots)]
    return Server(ss, budget, clock=clk), clk


def test_every_request_served_and_correct():
    reqs = make_requests(60)
    srv, _ = server()
    comps = srv.run(reqs)
    assert [c.rid for c in comps] == list(range(60))
    for r, c in zip(reqs, comps):
        assert c.ok, c.error
        lab, ap, nb = oracle_solve(r.graph)
        assert np.array_equal(c.edge_label, lab) and np.array_equal(c.is_ap, ap) and c.num_bcc == nb
        assert c.finished >= c.admitted >= c.arrival
    assert srv.stats["admitted"] == 60


def test_continuous_batching_joins_requests_that_arrive_while_busy():
    # slow slot: requests arriving during a batch are packed into the next one
    reqs = make_requests(40, qps=20000.0)
    srv, _ = server(slots=1, cost=lambda gs: 5e-3)
    comps = srv.run(reqs)
    assert all(c.ok for c in comps)
    assert srv.stats["batches"] < 40  # batched, not one by one
    assert srv.stats["max_queue"] > 1


def test_memory_budget_blocks_then_admits():
    reqs = make_requests(20, qps=1e6)
    one = max(request_bytes(int(r.graph.n), int(r.graph.offsets[-1])) for r in reqs)
    srv, _ = server(slots=4, budget=one + 1, cost=lambda gs: 1e-3)
    comps = srv.run(reqs)
    assert all(c.ok for c in comps)
    assert srv.stats["blocked_on_memory"] > 0
    assert srv.stats["max_inflight_bytes"] <= one + 1


def test_bad_and_oversized_requests_are_isolated():
    reqs = make_requests(12)
    bad = gen.Csr(3, np.array([0, 1, 2, 2], np.int64), np.array([1, 9], np.int32))  # id out of range
    big = gen.from_edges(5000, [(i, i + 1) for i in range(4999)])
    reqs[3] = Request(3, bad, reqs[3].arrival)
    reqs[7] = Request(7, big, reqs[7].arrival)
    srv, _ = server(cap_v=4000, cap_a=30000)
    comps = srv.run(reqs)
    assert not comps[3].ok and "range" in comps[3].error
    assert not comps[7].ok and "slot" in comps[7].error
    assert all(c.ok for i, c in enumerate(comps) if i not in (3, 7))
    assert srv.stats["rejected"] == 2


def test_request_over_budget_rejected_not_stuck():
    reqs = make_requests(5)
    srv, _ = server(budget=1000)
    comps = srv.run(reqs)
    assert all((not c.ok) and "budget" in c.error for c in comps)


def test_latency_summary():
    reqs = make_requests(30)
    srv, _ = server()
    s = latency_summary(srv.run(reqs))
    assert 0 < s["p50_ms"] <= s["p99_ms"] and s["graphs_per_s"] > 0


def test_serving_flags_are_the_serving_slot_pick():
    """Serving slots run their own shipped pick (a batch of a few large
    requests), not the 4096-graph batch's, whose per-graph passes give each
    graph one workgroup; and under the general input contract (no promises)."""
    from paper_2301_01356_amd import _native as N
    from paper_2301_01356_amd import tune
    from paper_2301_01356_amd.serve import serving_flags

    entries = tune.shipped_entries()
    assert serving_flags() == entries["serve8"][0]
    assert entries["serve8"][1]["tuned_on"] == "serve8"
    assert serving_flags() & (N.FLAG_SORTED_ROWS | N.FLAG_NO_SELF_LOOPS | N.FLAG_VALIDATE) == 0
