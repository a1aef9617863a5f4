"""Serving: continuous batching of BCC requests on one GPU.

Requests (host CSR graphs) arrive over time.  The scheduler keeps a FIFO
queue and a set of executor slots; whenever a slot is free it admits the
longest prefix of the queue that fits (a) the slot's vertex/arc/graph
capacity and (b) the HBM budget still free, packs those graphs into one batch
and launches it.  Requests that arrive while other batches are on the GPU
join the next batch as soon as a slot and memory free up; several slots
(each with its own HIP stream and device-resident buffers) keep copies and
kernels of different batches overlapping on the device.

Malformed requests are rejected at admission (status set on that request
only); an oversized request that no slot can hold is rejected the same way.
Latency is measured from arrival to the result being on the host.

The slot interface is small so the scheduler runs unchanged against
``HipSlot`` (the GPU) or ``SimSlot`` (any host solver + a simulated clock),
which is how admission, backpressure and error isolation are tested on CPU.
"""
from __future__ import annotations

import time
from dataclasses import dataclass
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np


@dataclass
class Request:
    rid: int
    graph: object  # .n, .offsets (int64/int32 [n+1]), .adj (int32)
    arrival: float  # seconds on the server clock


@dataclass
class Completion:
    rid: int
    ok: bool
    error: str = ""
    edge_label: Optional[np.ndarray] = None
    is_ap: Optional[np.ndarray] = None
    num_bcc: int = -1
    arrival: float = 0.0
    admitted: float = 0.0
    finished: float = 0.0

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def request_bytes(n: int, arcs: int) -> int:
    """Device bytes a request occupies inside a batch: its share of the
    workspace (O(n) plus tile bookkeeping) and its input/output arrays."""
    from . import _native as N

    return N.workspace_size(n, arcs, 1) + 4 * (n + 1) + 4 * arcs + 4 * arcs + n


def check_request(g) -> str:
    """Cheap host-side validation; returns an error string or ''."""
    try:
        n = int(g.n)
        off = np.asarray(g.offsets)
        adj = np.asarray(g.adj)
    except Exception as e:  # pragma: no cover - defensive
        return f"unreadable request: {e}"
    if n < 0 or off.shape != (n + 1,):
        return "offsets must have n + 1 entries"
    if off[0] != 0 or int(off[-1]) != adj.shape[0]:
        return "offsets must start at 0 and end at the arc count"
    if n and np.any(np.diff(off) < 0):
        return "offsets must be nondecreasing"
    if adj.size and (int(adj.min()) < 0 or int(adj.max()) >= n):
        return "vertex id out of range"
    if adj.size >= 2**31 or n >= 2**30:
        return "graph too large"
    return ""


class Slot:
    """Executor-side unit that runs one batch at a time."""

    cap_v: int
    cap_a: int
    cap_g: int

    def launch(self, graphs: Sequence) -> None: ...
    def ready(self) -> bool: ...
    def results(self) -> list: ...

    def eta(self) -> Optional[float]:
        """Clock time at which the running batch completes, if known."""
        return None


class Clock:
    def now(self) -> float:
        return time.perf_counter()

    def sleep_until(self, t: float) -> None:
        d = t - self.now()
        if d > 0:
            time.sleep(min(d, 0.0005))


@dataclass
class _Inflight:
    slot: int
    reqs: List[Request]
    bytes: int
    admitted: float


class Server:
    def __init__(self, slots: Sequence[Slot], hbm_budget: int, clock: Optional[Clock] = None,
                 max_batch_graphs: Optional[int] = None, on_idle: Optional[Callable[[], None]] = None):
        self.slots = list(slots)
        self.budget = int(hbm_budget)
        self.clock = clock or Clock()
        self.max_batch = max_batch_graphs
        self.on_idle = on_idle
        self.stats: Dict[str, int] = {"batches": 0, "admitted": 0, "rejected": 0, "max_queue": 0,
                                      "blocked_on_memory": 0, "max_inflight_bytes": 0}

    def _fits_any_slot(self, g) -> bool:
        n, a = int(g.n), int(g.offsets[-1])
        return any(n + 1 <= s.cap_v and a <= s.cap_a for s in self.slots)

    def run(self, requests: Sequence[Request]) -> List[Completion]:
        """Serve requests with the given arrival times; returns completions in
        request order."""
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        queue: List[Request] = []
        free = list(range(len(self.slots)))
        inflight: Dict[int, _Inflight] = {}
        used = 0
        done: Dict[int, Completion] = {}
        i = 0
        t0 = self.clock.now()
        while i < len(pending) or queue or inflight:
            now = self.clock.now() - t0
            # arrivals
            while i < len(pending) and pending[i].arrival <= now:
                r = pending[i]
                i += 1
                err = check_request(r.graph)
                if not err and not self._fits_any_slot(r.graph):
                    err = "request larger than any slot"
                if err:
                    done[r.rid] = Completion(r.rid, False, err, arrival=r.arrival, admitted=now, finished=now)
                    self.stats["rejected"] += 1
                else:
                    queue.append(r)
            self.stats["max_queue"] = max(self.stats["max_queue"], len(queue))
            # completions
            for si in list(inflight):
                fl = inflight[si]
                if self.slots[si].ready():
                    res = self.slots[si].results()
                    fin = self.clock.now() - t0
                    for r, gr in zip(fl.reqs, res):
                        done[r.rid] = Completion(r.rid, True, "", gr.edge_label, gr.is_ap, gr.num_bcc,
                                                 r.arrival, fl.admitted, fin)
                    used -= fl.bytes
                    del inflight[si]
                    free.append(si)
            # admission: FIFO prefix that fits a free slot and the budget
            while free and queue:
                head = queue[0]
                nh, ah = int(head.graph.n), int(head.graph.offsets[-1])
                if request_bytes(nh, ah) > self.budget:
                    queue.pop(0)
                    done[head.rid] = Completion(head.rid, False, "request exceeds the memory budget",
                                                arrival=head.arrival, admitted=now, finished=now)
                    self.stats["rejected"] += 1
                    continue
                cand = [k for k in free if nh + 1 <= self.slots[k].cap_v and ah <= self.slots[k].cap_a]
                if not cand:
                    break  # a slot big enough is busy: wait for it
                si = cand[0]
                s = self.slots[si]
                batch, nv, na, nbytes = [], 0, 0, 0
                for r in queue:
                    n, a = int(r.graph.n), int(r.graph.offsets[-1])
                    b = request_bytes(n, a)
                    if (nv + n + 1 > s.cap_v or na + a > s.cap_a or len(batch) + 1 > s.cap_g
                            or (self.max_batch and len(batch) + 1 > self.max_batch)
                            or used + nbytes + b > self.budget):
                        break
                    batch.append(r)
                    nv, na, nbytes = nv + n, na + a, nbytes + b
                if not batch:
                    self.stats["blocked_on_memory"] += 1
                    break  # only in-flight batches hold the memory it needs
                del queue[: len(batch)]
                free.remove(si)
                adm = self.clock.now() - t0
                s.launch([r.graph for r in batch])
                inflight[si] = _Inflight(si, batch, nbytes, adm)
                used += nbytes
                self.stats["max_inflight_bytes"] = max(self.stats["max_inflight_bytes"], used)
                self.stats["batches"] += 1
                self.stats["admitted"] += len(batch)
            # wait for the next arrival or completion
            wake = []
            if i < len(pending):
                wake.append(pending[i].arrival + t0)
            etas = [self.slots[k].eta() for k in inflight]
            if inflight and all(e is not None for e in etas):
                wake.extend(etas)
            elif inflight:
                wake.append(self.clock.now())  # real slots: poll
            if wake:
                if self.on_idle:
                    self.on_idle()
                self.clock.sleep_until(min(wake))
        return [done[r.rid] for r in sorted(requests, key=lambda r: r.rid)]


def latency_summary(comps: Sequence[Completion]) -> Dict[str, float]:
    lat = np.array([c.latency for c in comps if c.ok], dtype=np.float64)
    if lat.size == 0:
        return {"p50_ms": float("nan"), "p99_ms": float("nan"), "mean_ms": float("nan"), "graphs_per_s": 0.0}
    span = max(c.finished for c in comps if c.ok) - min(c.arrival for c in comps if c.ok)
    return {
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3),
        "graphs_per_s": float(lat.size / span) if span > 0 else float("inf"),
    }


def poisson_arrivals(count: int, qps: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / qps, size=count))


# ---------------------------------------------------------------- executors
class HipSlot(Slot):
    """A BatchedSolver with its own stream and device-resident buffers."""

    def __init__(self, cap_v: int, cap_a: int, cap_g: int, device="cuda:0", flags: int = 0, use_graph: bool = True):
        from .batch import BatchedSolver

        self.cap_v, self.cap_a, self.cap_g = cap_v, cap_a, cap_g
        self.solver = BatchedSolver(cap_v, cap_a, cap_g, device=device, flags=flags, use_graph=use_graph)

    def launch(self, graphs):
        self.solver.stage(graphs)
        self.solver.launch()

    def ready(self):
        return self.solver.ready()

    def results(self):
        return self.solver.results()


def hip_slots(num_slots: int, cap_v: int, cap_a: int, cap_g: int, device="cuda:0", flags: int = 0,
              use_graph: bool = True) -> List[HipSlot]:
    return [HipSlot(cap_v, cap_a, cap_g, device, flags, use_graph) for _ in range(num_slots)]


class SimClock(Clock):
    """Simulated clock for CPU tests: time advances only when waited on."""

    def __init__(self):
        self.t = 0.0

    def now(self) -> float:
        return self.t

    def sleep_until(self, t: float) -> None:
        self.t = max(self.t, t)


class SimSlot(Slot):
    """CPU stand-in for a GPU slot: solves with a given function and takes
    ``cost(graphs)`` simulated seconds from launch to ready."""

    def __init__(self, clock: SimClock, solve_fn, cap_v: int, cap_a: int, cap_g: int, cost=None):
        self.clock, self.solve_fn = clock, solve_fn
        self.cap_v, self.cap_a, self.cap_g = cap_v, cap_a, cap_g
        self.cost = cost or (lambda gs: 1e-3 + 1e-9 * sum(int(g.offsets[-1]) for g in gs))
        self.t_ready = None
        self.graphs = None

    def launch(self, graphs):
        assert self.t_ready is None, "slot launched while busy"
        self.graphs = list(graphs)
        self.t_ready = self.clock.now() + self.cost(self.graphs)

    def ready(self):
        return self.t_ready is not None and self.clock.now() >= self.t_ready

    def eta(self):
        return self.t_ready

    def results(self):
        from .batch import GraphResult

        out = []
        for g in self.graphs:
            lab, ap, nb = self.solve_fn(g)
            out.append(GraphResult(lab, ap, nb))
        self.t_ready = None
        self.graphs = None
        return out
