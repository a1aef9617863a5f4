"""Batched solving: many graphs, one launch sequence.

A batch is a disjoint union of graphs in one CSR (graph g owns a contiguous
vertex range; its arcs hold global ids).  ``fastbcc_solve_batched`` solves the
union in one launch sequence and returns graph-local labels.  This module
keeps device-resident buffers for a batch and moves only what a batch uses:

* host side, each graph's own CSR (graph-local ids) is copied into pinned
  staging memory, or, when the graph already lives in pinned memory
  (``PinnedGraph``), copied to the device straight from there;
* device side, the graph's vertex and arc offsets are added to its ids and
  row starts (``fastbcc_batch_rebase``).

Two modes:

* exact (``exact=True``): the batched solve runs eagerly on exactly the
  vertices, arcs and graphs of the batch -- what a serving slot does;
* fixed shape (default): the buffers always hold ``max_vertices`` vertices,
  ``max_arcs`` arcs and ``max_graphs + 1`` graphs, so the launch sequence can
  be captured once into a HIP graph (torch's CUDA-graph API drives
  hipStreamBeginCapture on ROCm) and replayed for every later batch.  The
  unused part is one padding graph: empty rows, and the unused arcs as
  parallel copies of one edge between its last two vertices (a 2-cycle: one
  BCC of its own, no articulation point), so the padding keeps rows sorted
  and free of self-loops; only an odd leftover arc becomes a self-loop.

The solve issues no host synchronisation and no memset, only kernels, which
is what makes it capturable.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _native as N
from .api import BccResult, alloc_workspace, batch_rebase, check_batched, greedy_packs, solve_batched, solve_small


@dataclass
class GraphResult:
    edge_label: Optional[np.ndarray]  # int32, graph-local arc ids (None when not kept)
    is_ap: Optional[np.ndarray]  # uint8
    num_bcc: int
    digest: Optional[int] = None  # device-side fingerprint of the labels and AP flags
    status: int = 0  # device input check of the graph (0 = passed; checked batches only)


class PinnedGraph:
    """A host CSR graph whose arrays live in pinned memory, so a batch copies
    it to the device without a staging copy (``.n``, ``.offsets``, ``.adj`` as
    numpy views of the pinned buffers, int32)."""

    def __init__(self, g):
        n, A = int(g.n), int(g.offsets[-1])
        self.n = n
        self.t_off = torch.empty(n + 1, dtype=torch.int32, pin_memory=True)
        self.t_adj = torch.empty(max(A, 1), dtype=torch.int32, pin_memory=True)[:A]
        self.offsets = self.t_off.numpy()
        self.adj = self.t_adj.numpy()
        self.offsets[:] = np.asarray(g.offsets)
        self.adj[:] = np.asarray(g.adj)

    @property
    def num_arcs(self) -> int:
        return int(self.adj.shape[0])


def pad_layout(used_v: int, used_a: int, cap_v: int, cap_a: int):
    """Where the padding graph puts the leftover arcs: (row start of vertex
    cap_v - 2, row start of vertex cap_v - 1, arcs per direction of the
    parallel edge, whether one self-loop closes an odd leftover)."""
    left = cap_a - used_a
    half = left // 2
    return used_a, used_a + half, half, bool(left & 1)


def pack(graphs: Sequence, max_vertices: int, max_arcs: int, max_graphs: int):
    """The padded union on the host (what the fixed-shape device buffers hold
    after a batch is staged): (vbegin int32[max_graphs+2], offsets
    int32[max_vertices+1], adj int32[max_arcs], per-graph (v0, v1, a0, a1))."""
    G = len(graphs)
    if G > max_graphs:
        raise ValueError(f"{G} graphs exceed the capacity {max_graphs}")
    nv = sum(int(g.n) for g in graphs)
    na = sum(int(g.offsets[-1]) for g in graphs)
    spare = 2 if na < max_arcs else 1
    if nv > max_vertices - spare or na > max_arcs:
        raise ValueError("batch exceeds the vertex/arc capacity")
    vbegin = np.zeros(max_graphs + 2, np.int32)
    offsets = np.empty(max_vertices + 1, np.int32)
    adj = np.empty(max_arcs, np.int32)
    v0 = a0 = 0
    spans = []
    for i, g in enumerate(graphs):
        n, A = int(g.n), int(g.offsets[-1])
        vbegin[i] = v0
        offsets[v0 : v0 + n] = np.asarray(g.offsets[:n], np.int64) + a0
        adj[a0 : a0 + A] = np.asarray(g.adj, np.int32) + v0
        spans.append((v0, v0 + n, a0, a0 + A))
        v0 += n
        a0 += A
    vbegin[G : max_graphs + 1] = v0
    vbegin[max_graphs + 1] = max_vertices
    r2, r1, half, odd = pad_layout(v0, a0, max_vertices, max_arcs)
    offsets[v0:max_vertices] = a0
    if max_arcs > a0:
        offsets[max_vertices - 1] = r1
        adj[r2:r1] = max_vertices - 1
        adj[r1 : r1 + half] = max_vertices - 2
        if odd:
            adj[max_arcs - 1] = max_vertices - 1
    offsets[max_vertices] = max_arcs
    return vbegin, offsets, adj, spans


def device_digests(label: torch.Tensor, is_ap: torch.Tensor, abound: torch.Tensor, vbound: torch.Tensor):
    """Per-graph fingerprint, computed on the device, of graph-local labels
    and AP flags of consecutive graphs (arc and vertex bounds int64[G+1]):
    sum over the graph's arcs of (label + 2) * (local arc index + 1) plus
    sum over its vertices of ap * (local vertex index + 1), in wrapping
    int64 arithmetic.  Equal results give equal digests; the serving
    benchmark compares them between served and serial solves."""
    dev = label.device

    def seg(vals: torch.Tensor, bound: torch.Tensor):
        m = vals.numel()
        idx = torch.arange(1, m + 1, dtype=torch.int64, device=dev)
        c1 = torch.zeros(m + 1, dtype=torch.int64, device=dev)
        c0 = torch.zeros(m + 1, dtype=torch.int64, device=dev)
        torch.cumsum(vals * idx, 0, out=c1[1:])
        torch.cumsum(vals, 0, out=c0[1:])
        lo, hi = bound[:-1], bound[1:]
        # sum (x) * (global + 1) - start * sum (x) = sum (x) * (local + 1)
        return (c1[hi] - c1[lo]) - lo * (c0[hi] - c0[lo])

    return seg(label.to(torch.int64) + 2, abound) + seg(is_ap.to(torch.int64), vbound)


class BatchedSolver:
    """Device-resident batch buffers, exact or fixed-shape (HIP-graph replay).

    ``small=True`` solves with the fused small-graph kernels
    (``fastbcc_solve_small``) instead of the general batched path: graphs of
    at most ``N.SMALL_MAX_VERTICES`` vertices, packed greedily into runs of
    at most ``pack_vertices`` vertices, no workspace."""

    def __init__(self, max_vertices: int, max_arcs: int, max_graphs: int, device="cuda:0", flags: int = 0,
                 use_graph: bool = True, stream: Optional[torch.cuda.Stream] = None, exact: bool = False,
                 digests: bool = False, check: bool = False, small: bool = False,
                 pack_vertices: int = N.SMALL_MAX_VERTICES):
        self.cap_v, self.cap_a, self.cap_g = int(max_vertices), int(max_arcs), int(max_graphs)
        self.device = torch.device(device)
        self.flags = flags
        self.small = small
        self.pack_vertices = int(pack_vertices)
        self.exact = exact
        self.use_graph = use_graph and not exact
        self.digests = digests
        self.check = check and exact  # device input check (and repair) before every exact solve
        G1 = self.cap_g + 1  # + the padding graph
        dev = self.device
        self.d_vbegin = torch.empty(G1 + 1, dtype=torch.int32, device=dev)
        self.d_off = torch.empty(self.cap_v + 1, dtype=torch.int32, device=dev)
        self.d_adj = torch.empty(self.cap_a, dtype=torch.int32, device=dev)
        self.out = BccResult(
            torch.empty(self.cap_a, dtype=torch.int32, device=dev),
            torch.empty(self.cap_v, dtype=torch.uint8, device=dev),
            torch.empty(G1, dtype=torch.int64, device=dev),
        )
        self.ws = None if small else alloc_workspace(self.cap_v, self.cap_a, G1, dev)
        # pack starts (small mode): at most one pack per graph; unused packs
        # are empty, so a captured launch always covers cap_g + 1 packs
        self.h_packs = torch.zeros(G1 + 1, dtype=torch.int32, pin_memory=True)
        self.d_packs = torch.zeros(G1 + 1, dtype=torch.int32, device=dev)
        self.num_packs = 0
        # pinned staging for host<->device copies
        self.h_vbegin = torch.empty(G1 + 1, dtype=torch.int32, pin_memory=True)
        self.h_bounds = torch.empty(2 * (G1 + 1), dtype=torch.int64, pin_memory=True)
        self.h_abegin = torch.empty(G1 + 1, dtype=torch.int32, pin_memory=True)
        self.d_abegin = torch.empty(G1 + 1, dtype=torch.int32, device=dev)
        self._h_in = None  # pinned staging of graphs that are not pinned themselves (allocated on first use)
        self.h_label = torch.empty(self.cap_a, dtype=torch.int32, pin_memory=True)
        self.h_ap = torch.empty(self.cap_v, dtype=torch.uint8, pin_memory=True)
        self.h_nb = torch.empty(G1, dtype=torch.int64, pin_memory=True)
        self.h_dig = torch.empty(G1, dtype=torch.int64, pin_memory=True)
        self.d_status = torch.zeros(G1, dtype=torch.int32, device=dev)
        self.h_status = torch.zeros(G1, dtype=torch.int32, pin_memory=True)
        self.stream = stream or torch.cuda.Stream(device=dev)
        self.graph: Optional[torch.cuda.CUDAGraph] = None
        self.done = torch.cuda.Event()
        self.spans: List[tuple] = []
        self._copies: List[tuple] = []
        self._keep_host = True
        # the device buffers always hold a valid (padded) CSR: start with the
        # empty batch so no launch can ever read uninitialised memory
        self.stage([])
        self._copy_in()
        self.stream.synchronize()

    @staticmethod
    def bytes_needed(max_vertices: int, max_arcs: int, max_graphs: int, small: bool = False) -> int:
        ws = 0 if small else N.workspace_size(max_vertices, max_arcs, max_graphs + 1)
        return ws + 2 * 4 * max_arcs + 5 * max_vertices + 8 * (max_graphs + 2) + 4 * (max_graphs + 2)

    # ------------------------------------------------------------ staging
    def stage(self, graphs: Sequence) -> None:
        """Lay the graphs out for the next launch: per graph its vertex and
        arc range; its CSR is copied into pinned staging now unless it lives
        in pinned memory already (then the launch copies it from there)."""
        G = len(graphs)
        if G > self.cap_g:
            raise ValueError(f"{G} graphs exceed the capacity {self.cap_g}")
        spans, copies = [], []
        v0 = a0 = 0
        for g in graphs:
            n, A = int(g.n), int(g.offsets[-1])
            spans.append((v0, v0 + n, a0, a0 + A))
            v0 += n
            a0 += A
        spare = 0 if self.exact else (2 if a0 < self.cap_a else 1)
        if v0 > self.cap_v - spare or a0 > self.cap_a:
            raise ValueError("batch exceeds the vertex/arc capacity")
        if self.small:
            too_big = [s1 - s0 for (s0, s1, _, _) in spans if s1 - s0 > N.SMALL_MAX_VERTICES]
            if too_big:
                raise ValueError(f"a graph of {too_big[0]} vertices exceeds the fused kernels' limit "
                                 f"{N.SMALL_MAX_VERTICES}")
            packs = greedy_packs([s1 - s0 for (s0, s1, _, _) in spans], self.pack_vertices)
            hp = self.h_packs.numpy()
            hp[: len(packs)] = packs
            hp[len(packs) :] = G
            self.num_packs = len(packs) - 1
        for g, (s0, s1, b0, b1) in zip(graphs, spans):
            if isinstance(g, PinnedGraph):
                copies.append((s0, s1, b0, b1, g.t_off, g.t_adj))
            else:
                hoff, hadj = self._staging()
                hoff[s0:s1] = np.asarray(g.offsets[: s1 - s0])
                hadj[b0:b1] = np.asarray(g.adj)
                copies.append((s0, s1, b0, b1, None, None))
        vb = self.h_vbegin.numpy()
        vb[:G] = [s[0] for s in spans]
        vb[G : self.cap_g + 1] = v0
        vb[self.cap_g + 1] = self.cap_v
        bd = self.h_bounds.numpy()
        bd[: G + 1] = [s[2] for s in spans] + [a0]
        bd[G + 1 : 2 * G + 2] = [s[0] for s in spans] + [v0]
        self.h_abegin.numpy()[: G + 1] = bd[: G + 1]
        self.spans, self._copies = spans, copies
        self.used_v, self.used_a = v0, a0

    def _staging(self):
        if self._h_in is None:
            self._h_in = (torch.empty(self.cap_v + 1, dtype=torch.int32, pin_memory=True),
                          torch.empty(self.cap_a, dtype=torch.int32, pin_memory=True))
        return self._h_in[0].numpy(), self._h_in[1].numpy()

    def _copy_in(self) -> None:
        """On this solver's stream: the staged graphs into the device buffers,
        their ids and offsets made global, and (fixed shape) the padding."""
        s = self.stream
        G, v0, a0 = len(self.spans), self.used_v, self.used_a
        with torch.cuda.stream(s):
            self.d_vbegin.copy_(self.h_vbegin, non_blocking=True)
            if self.small:
                self.d_packs.copy_(self.h_packs, non_blocking=True)
            # staged graphs sit contiguously in the staging buffers: copy each
            # run of them at once, pinned-source graphs one by one
            run = None
            for (s0, s1, b0, b1, toff, tadj) in self._copies + [(v0, v0, a0, a0, False, None)]:
                if toff is None:
                    run = (s0, b0) if run is None else run
                    continue
                if run is not None:
                    r0, rb = run
                    h_off, h_adj = self._h_in
                    if s0 > r0:
                        self.d_off[r0:s0].copy_(h_off[r0:s0], non_blocking=True)
                    if b0 > rb:
                        self.d_adj[rb:b0].copy_(h_adj[rb:b0], non_blocking=True)
                    run = None
                if toff is not False:
                    if s1 > s0:
                        self.d_off[s0:s1].copy_(toff[: s1 - s0], non_blocking=True)
                    if b1 > b0:
                        self.d_adj[b0:b1].copy_(tadj, non_blocking=True)
            if G:
                # graph-local -> global: each graph's first vertex added to its
                # arcs' targets, its first arc to its row starts (on the device)
                self.d_abegin[: G + 1].copy_(self.h_abegin[: G + 1], non_blocking=True)
                batch_rebase(self.d_off[: v0 + 1], self.d_adj[:a0], self.d_vbegin[: G + 1], self.d_abegin[: G + 1],
                             stream=s)
                if self.digests:
                    bd = self.h_bounds[: 2 * G + 2].to(self.device, non_blocking=True)
                    self._bounds = (bd[: G + 1], bd[G + 1 :])
            if self.exact:
                self.d_off[v0 : v0 + 1].fill_(a0)
            else:
                r2, r1, half, odd = pad_layout(v0, a0, self.cap_v, self.cap_a)
                self.d_off[v0 : self.cap_v].fill_(a0)
                self.d_off[self.cap_v : self.cap_v + 1].fill_(self.cap_a)
                if self.cap_a > a0:
                    self.d_off[self.cap_v - 1 : self.cap_v].fill_(r1)
                    self.d_adj[r2:r1].fill_(self.cap_v - 1)
                    self.d_adj[r1 : r1 + half].fill_(self.cap_v - 2)
                    if odd:
                        self.d_adj[self.cap_a - 1 :].fill_(self.cap_v - 1)

    # ------------------------------------------------------------ solving
    def _launch(self):
        if self.small:
            # promise bits only: the fused kernels take no tuning fields
            fl = self.flags & (N.FLAG_SORTED_ROWS | N.FLAG_NO_SELF_LOOPS)
            if self.exact:
                G, v, a = len(self.spans), self.used_v, self.used_a
                if G == 0 or self.num_packs == 0:
                    return
                out = BccResult(self.out.edge_label[:a], self.out.is_ap[:v], self.out.num_bcc[:G])
                solve_small(self.d_vbegin[: G + 1], self.d_off[: v + 1], self.d_adj[:a],
                            packs=self.d_packs[: self.num_packs + 1], out=out, flags=fl, stream=self.stream)
            else:
                solve_small(self.d_vbegin, self.d_off, self.d_adj, packs=self.d_packs, out=self.out, flags=fl,
                            stream=self.stream)
            return
        if self.exact:
            G, v, a = len(self.spans), self.used_v, self.used_a
            if G == 0:
                return
            if self.check:
                # untrusted graphs: checked on the device, failed ones made valid
                # in place, so the solve that follows is safe for the whole batch
                check_batched(self.d_off[: v + 1], self.d_adj[:a], self.d_vbegin[: G + 1], repair=True,
                              out=self.d_status[:G], stream=self.stream)
            out = BccResult(self.out.edge_label[:a], self.out.is_ap[:v], self.out.num_bcc[:G])
            solve_batched(self.d_vbegin[: G + 1], self.d_off[: v + 1], self.d_adj[:a], out=out, workspace=self.ws,
                          flags=self.flags, stream=self.stream)
        else:
            solve_batched(self.d_vbegin, self.d_off, self.d_adj, out=self.out, workspace=self.ws, flags=self.flags,
                          stream=self.stream)

    def _ensure_graph(self):
        if not self.use_graph or self.graph is not None:
            return
        with torch.cuda.stream(self.stream):
            # one eager run first (also warms the code objects), then capture
            self._launch()
            self.stream.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=self.stream):
                self._launch()
        self.stream.synchronize()
        self.graph = g

    def launch(self, keep_host: bool = True) -> None:
        """Copy the staged batch in, solve, copy results out -- all
        asynchronous on this solver's stream; ``self.done`` marks the end.
        Inputs are copied BEFORE any solve (the first call in fixed-shape mode
        also runs one eager solve and captures the graph, both on the copied
        batch).  ``keep_host=False`` copies only the counts (and digests)
        back, not the labels and AP flags."""
        s = self.stream
        self._copy_in()
        self._ensure_graph()
        G, v, a = len(self.spans), self.used_v, self.used_a
        with torch.cuda.stream(s):
            if self.graph is not None:
                self.graph.replay()
            else:
                self._launch()
            if self.digests and G:
                ab, vbd = self._bounds
                dig = device_digests(self.out.edge_label[:a], self.out.is_ap[:v], ab, vbd)
                self.h_dig[:G].copy_(dig, non_blocking=True)
            if keep_host:
                if a:
                    self.h_label[:a].copy_(self.out.edge_label[:a], non_blocking=True)
                if v:
                    self.h_ap[:v].copy_(self.out.is_ap[:v], non_blocking=True)
            if G:
                self.h_nb[:G].copy_(self.out.num_bcc[:G], non_blocking=True)
                if self.check:
                    self.h_status[:G].copy_(self.d_status[:G], non_blocking=True)
            self.done.record(s)
        self._keep_host = keep_host

    def ready(self) -> bool:
        return self.done.query()

    def results(self, copy: bool = True) -> List[GraphResult]:
        """Per-graph results of the last launch.  ``copy=False`` returns views
        of the pinned host buffers, valid until the next launch."""
        self.done.synchronize()
        lab = self.h_label.numpy()
        ap = self.h_ap.numpy()
        nb = self.h_nb.numpy()
        dig = self.h_dig.numpy()
        out = []
        for i, (v0, v1, a0, a1) in enumerate(self.spans):
            if self._keep_host:
                gl, ga = lab[a0:a1], ap[v0:v1]
                if copy:
                    gl, ga = gl.copy(), ga.copy()
            else:
                gl = ga = None
            out.append(GraphResult(gl, ga, int(nb[i]), int(dig[i]) if self.digests else None,
                                   int(self.h_status[i]) if self.check else 0))
        return out

    def solve(self, graphs: Sequence) -> List[GraphResult]:
        self.stage(graphs)
        self.launch()
        return self.results()


class SplitBatchedSolver:
    """A batch split by graph size: graphs of at most ``small_max``
    vertices go, packed, to the fused small-graph kernels, the others to the
    general batched path.  The two parts have their own buffers and streams,
    so their launches (or HIP-graph replays) overlap on the device; results
    come back in the order the graphs were staged."""

    def __init__(self, small_caps, big_caps, small_max: int = N.SMALL_MAX_VERTICES,
                 pack_vertices: int = N.SMALL_MAX_VERTICES, device="cuda:0", flags: int = 0, use_graph: bool = True):
        if not 0 <= small_max <= N.SMALL_MAX_VERTICES:
            raise ValueError(f"small_max must lie in [0, {N.SMALL_MAX_VERTICES}]")
        self.small_max = int(small_max)
        self.small = BatchedSolver(*small_caps, device=device, use_graph=use_graph, small=True,
                                   pack_vertices=pack_vertices)
        self.big = BatchedSolver(*big_caps, device=device, flags=flags, use_graph=use_graph)
        self.order: List[tuple] = []

    @staticmethod
    def capacities(graphs: Sequence, small_max: int = N.SMALL_MAX_VERTICES):
        """(vertices, arcs, graphs) capacities of the small and the big part
        for exactly these graphs (the big part's padding needs two spare
        vertices)."""
        sv = sa = sg = bv = ba = bg = 0
        for g in graphs:
            n, A = int(g.n), int(g.offsets[-1])
            if n <= small_max:
                sv, sa, sg = sv + n, sa + A, sg + 1
            else:
                bv, ba, bg = bv + n, ba + A, bg + 1
        return (sv + 2, max(sa, 1), max(sg, 1)), (bv + 2, max(ba, 1), max(bg, 1))

    @property
    def flags(self) -> int:
        return self.big.flags

    @flags.setter
    def flags(self, value: int) -> None:
        self.big.flags = value
        self.small.flags = value

    def stage(self, graphs: Sequence) -> None:
        """Split the graphs; the small ones are staged in decreasing size, so
        greedy packing fills nearly every pack to the largest class (a pack
        left small would get a launch of a smaller class to itself)."""
        small_idx, big, order = [], [], []
        for i, g in enumerate(graphs):
            if int(g.n) <= self.small_max:
                order.append(None)
                small_idx.append(i)
            else:
                order.append((1, len(big)))
                big.append(g)
        small_idx.sort(key=lambda i: -int(graphs[i].n))
        for k, i in enumerate(small_idx):
            order[i] = (0, k)
        self.small.stage([graphs[i] for i in small_idx])
        self.big.stage(big)
        self.order = order

    def launch(self, keep_host: bool = True) -> None:
        self.small.launch(keep_host)
        self.big.launch(keep_host)

    def replay(self) -> None:
        """Solve both parts again, each on its own stream, from their captured
        HIP graphs when they have them (inputs as last copied; nothing copied
        back)."""
        for part in (self.small, self.big):
            part._ensure_graph()
        for part in (self.small, self.big):
            with torch.cuda.stream(part.stream):
                if part.graph is not None:
                    part.graph.replay()
                else:  # built without HIP graphs: the same launches, eagerly
                    part._launch()

    def synchronize(self) -> None:
        self.small.stream.synchronize()
        self.big.stream.synchronize()

    def results(self, copy: bool = True) -> List[GraphResult]:
        parts = (self.small.results(copy), self.big.results(copy))
        return [parts[p][i] for p, i in self.order]

    def solve(self, graphs: Sequence) -> List[GraphResult]:
        self.stage(graphs)
        self.launch()
        return self.results()
