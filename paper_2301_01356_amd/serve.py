"""Serving: continuous batching of BCC requests on one GPU.

Requests (host CSR graphs) arrive over time.  The scheduler keeps a FIFO
queue and a set of executor slots; whenever a slot is free it admits the
longest prefix of the queue that fits (a) the slot's vertex/arc/graph
capacity and (b) the HBM budget still free, packs those graphs into one batch
and launches it.  Requests that arrive while other batches are on the GPU
join the next batch as soon as a slot and memory free up; several slots
(each with its own HIP stream and device-resident buffers) keep copies and
kernels of different batches overlapping on the device.  The budget is
re-read from the live free HBM (``free_hbm``) whenever a slot completes.

Slots solve under the general input contract (rows in any order, self-loops
allowed): a request is not trusted to keep the sorted-row or loop-free
promises.  Admission checks a request's sizes only (O(1) on the host); its
rows and ids are checked on the device, in the batch, before the solve
(fastbcc_check_batched): a graph that fails is made valid in place, solved
harmlessly with the others and reported as rejected.

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
    digest: Optional[int] = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def serving_flags() -> int:
    """Flags of the serving slots: the tuning fields shipped for a serving
    slot's batch (a few requests of up to 2^22 vertices each, under the
    general input contract).  The 4096-graph batch's pick does not carry
    over: its per-graph union-find passes suit many small graphs, not a few
    large ones."""
    from . import tune

    return tune.shipped_entries()["serve8"][0]


def request_bytes(n: int, arcs: int) -> int:
    """Device bytes a request occupies inside a batch: its share of the
    workspace (O(n) plus tile bookkeeping) and its input/output arrays."""
    from . import _native as N

    return N.workspace_size(n, arcs, 1) + 4 * (n + 1) + 4 * arcs + 4 * arcs + n


def check_request(g) -> str:
    """Host-side admission check, O(1): sizes and the two ends of the offsets
    (which place the request inside a batch).  Rows and ids are checked on
    the device with the batch."""
    try:
        n = int(g.n)
        off = g.offsets
        A = int(len(g.adj))
        if len(off) != n + 1:
            return "offsets must have n + 1 entries"
        first, last = int(off[0]), int(off[n])
    except Exception as e:  # pragma: no cover - defensive
        return f"unreadable request: {e}"
    if n < 0:
        return "negative vertex count"
    if first != 0 or last != A:
        return "offsets must start at 0 and end at the arc count"
    if A >= 2**31 or n >= 2**30:
        return "graph too large"
    return ""


def host_graph_status(g) -> int:
    """What the device input check reports for one graph, computed on the
    host (for the simulated slots of the CPU tests): 0 if every row lies
    inside the graph with nondecreasing offsets and every id is in range."""
    off = np.asarray(g.offsets, np.int64)
    adj = np.asarray(g.adj, np.int64)
    n = int(g.n)
    if n and np.any(np.diff(off) < 0):
        return 5
    if adj.size and (int(adj.min()) < 0 or int(adj.max()) >= n):
        return 5
    return 0


INVALID_GRAPH_ERROR = "invalid graph: a row outside the graph, decreasing offsets or an id out of range"


class Slot:
    """Executor-side unit that runs one batch at a time."""

    cap_v: int
    cap_a: int
    cap_g: int

    def launch(self, graphs: Sequence, keep: Optional[Sequence[bool]] = None) -> None: ...
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
    """``hbm_budget``: bytes the in-flight requests may hold.  ``free_hbm``
    (optional): a function returning the device's free bytes now; the budget
    is then re-read at every completion as what the in-flight batches hold
    plus ``hbm_fraction`` of the free bytes (capped by ``hbm_budget``).
    ``keep(request)`` decides whether a completion keeps the labels and AP
    flags on the host (default: always); the BCC count and, when the slot
    computes one, a device-side digest of the result are always kept."""

    def __init__(self, slots: Sequence[Slot], hbm_budget: int, clock: Optional[Clock] = None,
                 max_batch_graphs: Optional[int] = None, on_idle: Optional[Callable[[], None]] = None,
                 free_hbm: Optional[Callable[[], int]] = None, hbm_fraction: float = 0.6,
                 keep: Optional[Callable[[Request], bool]] = None):
        self.slots = list(slots)
        self.cap_budget = int(hbm_budget)
        self.budget = int(hbm_budget)
        self.clock = clock or Clock()
        self.max_batch = max_batch_graphs
        self.on_idle = on_idle
        self.free_hbm = free_hbm
        self.hbm_fraction = hbm_fraction
        self.keep = keep
        self.stats: Dict[str, int] = {"batches": 0, "admitted": 0, "rejected": 0, "max_queue": 0,
                                      "blocked_on_memory": 0, "max_inflight_bytes": 0, "budget_reads": 0,
                                      "min_budget": int(hbm_budget)}

    def _reread_budget(self, used: int) -> None:
        if self.free_hbm is None:
            return
        live = used + int(self.hbm_fraction * max(int(self.free_hbm()), 0))
        self.budget = min(self.cap_budget, live)
        self.stats["budget_reads"] += 1
        self.stats["min_budget"] = min(self.stats["min_budget"], self.budget)

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
        self._reread_budget(0)
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
                        if getattr(gr, "status", 0) != 0:
                            done[r.rid] = Completion(r.rid, False, INVALID_GRAPH_ERROR, arrival=r.arrival,
                                                     admitted=fl.admitted, finished=fin)
                            self.stats["rejected"] += 1
                            continue
                        kept = self.keep is None or self.keep(r)
                        lab = ap = None
                        if kept and gr.edge_label is not None:  # slots may hand out views of reused buffers
                            lab, ap = np.array(gr.edge_label, copy=True), np.array(gr.is_ap, copy=True)
                        done[r.rid] = Completion(r.rid, True, "", lab, ap, gr.num_bcc, r.arrival, fl.admitted,
                                                 fin, getattr(gr, "digest", None))
                    used -= fl.bytes
                    del inflight[si]
                    free.append(si)
                    self._reread_budget(used)
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
                s.launch([r.graph for r in batch], keep=[self.keep is None or self.keep(r) for r in batch])
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
    """A batched solver with its own stream and device-resident buffers; it
    solves each batch eagerly on exactly the batch's vertices and arcs."""

    def __init__(self, cap_v: int, cap_a: int, cap_g: int, device="cuda:0", flags: int = 0, digests: bool = False):
        from .batch import BatchedSolver

        self.cap_v, self.cap_a, self.cap_g = cap_v, cap_a, cap_g
        self.solver = BatchedSolver(cap_v, cap_a, cap_g, device=device, flags=flags, exact=True, digests=digests,
                                    check=True)

    def launch(self, graphs, keep=None):
        # results always travel to pinned host memory (a request's latency
        # ends there); ``keep`` only decides which ones the server copies out
        self.solver.stage(graphs)
        self.solver.launch()

    def ready(self):
        return self.solver.ready()

    def results(self):
        # views of the pinned result buffers (valid until this slot's next
        # launch): the server copies out only the results it keeps
        return self.solver.results(copy=False)


def hip_slots(num_slots: int, cap_v: int, cap_a: int, cap_g: int, device="cuda:0", flags: int = 0,
              digests: bool = False) -> List[HipSlot]:
    return [HipSlot(cap_v, cap_a, cap_g, device, flags, digests) for _ in range(num_slots)]


class PlainSlot(Slot):
    """Serial baseline: one request at a time through the plain solve
    (fastbcc_solve): the request's own CSR copied in, solved in a workspace
    sized for it, its labels and AP flags copied out -- nothing padded, no
    batching."""

    cap_g = 1

    def __init__(self, cap_v: int, cap_a: int, device="cuda:0", flags: int = 0, digests: bool = False):
        from .api import BccResult

        self.cap_v, self.cap_a = cap_v, cap_a
        self.device = torch_device(device)
        self.flags, self.digests = flags, digests
        import torch

        dev = self.device
        self.d_off = torch.empty(cap_v + 1, dtype=torch.int32, device=dev)
        self.d_adj = torch.empty(cap_a, dtype=torch.int32, device=dev)
        self.out = BccResult(torch.empty(cap_a, dtype=torch.int32, device=dev),
                             torch.empty(cap_v, dtype=torch.uint8, device=dev),
                             torch.empty(1, dtype=torch.int64, device=dev))
        self.h_off = torch.empty(cap_v + 1, dtype=torch.int32, pin_memory=True)
        self.h_adj = torch.empty(cap_a, dtype=torch.int32, pin_memory=True)
        self.h_label = torch.empty(cap_a, dtype=torch.int32, pin_memory=True)
        self.h_ap = torch.empty(cap_v, dtype=torch.uint8, pin_memory=True)
        self.h_nb = torch.empty(1, dtype=torch.int64, pin_memory=True)
        self.h_dig = torch.empty(1, dtype=torch.int64, pin_memory=True)
        self.d_status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.h_status = torch.zeros(1, dtype=torch.int32, pin_memory=True)
        self.h_bounds = torch.zeros(4, dtype=torch.int64, pin_memory=True)  # [0, A, 0, n] for the digest
        self.stream = torch.cuda.Stream(device=dev)
        self.done = torch.cuda.Event()
        self.n = self.a = 0
        self.kept = True

    def launch(self, graphs, keep=None):
        import numpy as np
        import torch

        from .api import BccResult, alloc_workspace, check_batched, solve
        from .batch import PinnedGraph, device_digests

        (g,) = graphs
        n, A = int(g.n), int(g.offsets[-1])
        if isinstance(g, PinnedGraph):
            src_off, src_adj = g.t_off, g.t_adj
        else:
            self.h_off.numpy()[: n + 1] = np.asarray(g.offsets)
            self.h_adj.numpy()[:A] = np.asarray(g.adj)
            src_off, src_adj = self.h_off[: n + 1], self.h_adj[:A]
        self.n, self.a = n, A
        self.kept = keep is None or keep[0]
        s = self.stream
        with torch.cuda.stream(s):
            self.d_off[: n + 1].copy_(src_off, non_blocking=True)
            if A:
                self.d_adj[:A].copy_(src_adj, non_blocking=True)
            # the request's rows and ids checked on the device first (a graph
            # that fails is made valid in place and its result dropped)
            check_batched(self.d_off[: n + 1], self.d_adj[:A], repair=True, out=self.d_status, stream=s)
            ws = alloc_workspace(n, A, 1, self.device)
            out = BccResult(self.out.edge_label[:A], self.out.is_ap[:n], self.out.num_bcc)
            solve(self.d_off[: n + 1], self.d_adj[:A], out=out, workspace=ws, flags=self.flags, stream=s)
            if self.digests:
                # bounds staged through pinned memory that stays untouched until
                # this request completes (a pageable source could be reused early)
                self.h_bounds.numpy()[:] = (0, A, 0, n)
                bd = self.h_bounds.to(self.device, non_blocking=True)
                self.h_dig.copy_(device_digests(out.edge_label, out.is_ap, bd[:2], bd[2:]), non_blocking=True)
            if A:
                self.h_label[:A].copy_(out.edge_label, non_blocking=True)
            if n:
                self.h_ap[:n].copy_(out.is_ap, non_blocking=True)
            self.h_nb.copy_(out.num_bcc, non_blocking=True)
            self.h_status.copy_(self.d_status, non_blocking=True)
            self.done.record(s)

    def ready(self):
        return self.done.query()

    def results(self):
        from .batch import GraphResult

        self.done.synchronize()
        lab = self.h_label.numpy()[: self.a].copy() if self.kept else None
        ap = self.h_ap.numpy()[: self.n].copy() if self.kept else None
        return [GraphResult(lab, ap, int(self.h_nb.numpy()[0]), int(self.h_dig.numpy()[0]) if self.digests else None,
                            int(self.h_status.numpy()[0]))]


def torch_device(device):
    import torch

    return torch.device(device)


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

    def launch(self, graphs, keep=None):
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
            st = host_graph_status(g)
            if st:
                out.append(GraphResult(None, None, -1, None, st))
                continue
            lab, ap, nb = self.solve_fn(g)
            out.append(GraphResult(lab, ap, nb))
        self.t_ready = None
        self.graphs = None
        return out
