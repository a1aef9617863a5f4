"""Batched solving: many graphs, one launch sequence, replayed as a HIP graph.

A batch is a disjoint union of graphs in one CSR (graph g owns a contiguous
vertex range; its arcs hold global ids).  ``fastbcc_solve_batched`` solves the
union in one launch sequence and returns graph-local labels; this module adds
fixed-capacity device buffers and captures that sequence once into a HIP
graph (torch's CUDA-graph API drives hipStreamBeginCapture on ROCm), so each
later batch costs one graph launch.  The solve issues no host synchronisation
and no memset, only kernels, which is what makes it capturable.

A batch smaller than the capacity is padded: one extra padding graph takes
the unused vertices, and its last vertex holds the unused arcs as self-loops
(label -1, no BCC, no articulation point), so the captured shapes never
change.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _native as N
from .api import BccResult, alloc_workspace, solve_batched


@dataclass
class GraphResult:
    edge_label: np.ndarray  # int32, graph-local arc ids
    is_ap: np.ndarray  # uint8
    num_bcc: int


def pack(graphs: Sequence, max_vertices: int, max_arcs: int, max_graphs: int):
    """Concatenate host CSR graphs (objects with .n, .offsets, .adj) into
    padded union arrays: (vbegin int32[max_graphs+2], offsets int32[max_vertices+1],
    adj int32[max_arcs], per-graph (vbegin, abegin))."""
    G = len(graphs)
    if G > max_graphs:
        raise ValueError(f"{G} graphs exceed the capacity {max_graphs}")
    nv = sum(int(g.n) for g in graphs)
    na = sum(int(g.offsets[-1]) for g in graphs)
    if nv > max_vertices - 1 or na > max_arcs:
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
    # padding graph(s): empty graphs up to max_graphs, then one graph holding
    # the remaining vertices; its last vertex carries the leftover arcs as loops
    vbegin[G : max_graphs + 1] = v0
    vbegin[max_graphs + 1] = max_vertices
    offsets[v0:max_vertices] = a0
    offsets[max_vertices - 1] = a0
    offsets[max_vertices] = max_arcs
    adj[a0:] = max_vertices - 1
    return vbegin, offsets, adj, spans


class BatchedSolver:
    """Fixed-capacity batched solver with optional HIP-graph replay."""

    def __init__(self, max_vertices: int, max_arcs: int, max_graphs: int, device="cuda:0", flags: int = 0,
                 use_graph: bool = True, stream: Optional[torch.cuda.Stream] = None):
        self.cap_v, self.cap_a, self.cap_g = int(max_vertices), int(max_arcs), int(max_graphs)
        self.device = torch.device(device)
        self.flags = flags
        self.use_graph = use_graph
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
        self.ws = alloc_workspace(self.cap_v, self.cap_a, G1, dev)
        # pinned staging for host<->device copies
        self.h_vbegin = torch.empty(G1 + 1, dtype=torch.int32, pin_memory=True)
        self.h_off = torch.empty(self.cap_v + 1, dtype=torch.int32, pin_memory=True)
        self.h_adj = torch.empty(self.cap_a, dtype=torch.int32, pin_memory=True)
        self.h_label = torch.empty(self.cap_a, dtype=torch.int32, pin_memory=True)
        self.h_ap = torch.empty(self.cap_v, dtype=torch.uint8, pin_memory=True)
        self.h_nb = torch.empty(G1, dtype=torch.int64, pin_memory=True)
        self.stream = stream or torch.cuda.Stream(device=dev)
        self.graph: Optional[torch.cuda.CUDAGraph] = None
        self.done = torch.cuda.Event()
        self.spans: List[tuple] = []
        # the device buffers always hold a valid (padded) CSR: start with the
        # empty batch so no launch can ever read uninitialised memory
        self.stage([])
        with torch.cuda.stream(self.stream):
            self.d_vbegin.copy_(self.h_vbegin, non_blocking=True)
            self.d_off.copy_(self.h_off, non_blocking=True)
            self.d_adj.copy_(self.h_adj, non_blocking=True)
        self.stream.synchronize()

    @staticmethod
    def bytes_needed(max_vertices: int, max_arcs: int, max_graphs: int) -> int:
        ws = N.workspace_size(max_vertices, max_arcs, max_graphs + 1)
        return ws + 2 * 4 * max_arcs + 5 * max_vertices + 8 * (max_graphs + 2) + 4 * (max_graphs + 2)

    def _launch(self):
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

    def stage(self, graphs: Sequence) -> None:
        """Pack host graphs into the pinned staging buffers."""
        vb, off, adj, spans = pack(graphs, self.cap_v, self.cap_a, self.cap_g)
        self.h_vbegin.numpy()[:] = vb
        self.h_off.numpy()[:] = off
        self.h_adj.numpy()[:] = adj
        self.spans = spans

    def launch(self) -> None:
        """Copy the staged batch in, solve, copy results out -- all
        asynchronous on this solver's stream; ``self.done`` marks the end.
        Inputs are copied BEFORE any solve (the first call also runs one eager
        solve and captures the graph, both on the copied batch)."""
        s = self.stream
        with torch.cuda.stream(s):
            self.d_vbegin.copy_(self.h_vbegin, non_blocking=True)
            self.d_off.copy_(self.h_off, non_blocking=True)
            used_a = self.spans[-1][3] if self.spans else 0
            if used_a:
                self.d_adj[:used_a].copy_(self.h_adj[:used_a], non_blocking=True)
            # padding arcs: self-loops on the last vertex (device fill)
            if used_a < self.cap_a:
                self.d_adj[used_a:].fill_(self.cap_v - 1)
        self._ensure_graph()
        with torch.cuda.stream(s):
            if self.graph is not None:
                self.graph.replay()
            else:
                self._launch()
            if used_a:
                self.h_label[:used_a].copy_(self.out.edge_label[:used_a], non_blocking=True)
            self.h_ap.copy_(self.out.is_ap, non_blocking=True)
            self.h_nb.copy_(self.out.num_bcc, non_blocking=True)
            self.done.record(s)

    def ready(self) -> bool:
        return self.done.query()

    def results(self) -> List[GraphResult]:
        self.done.synchronize()
        lab = self.h_label.numpy()
        ap = self.h_ap.numpy()
        nb = self.h_nb.numpy()
        out = []
        for i, (v0, v1, a0, a1) in enumerate(self.spans):
            out.append(GraphResult(lab[a0:a1].copy(), ap[v0:v1].copy(), int(nb[i])))
        return out

    def solve(self, graphs: Sequence) -> List[GraphResult]:
        self.stage(graphs)
        self.launch()
        return self.results()
