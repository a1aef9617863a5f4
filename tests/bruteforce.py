"""Biconnected components straight from their definitions, for tiny graphs.

Independent of both the oracle and the HIP path:

* Edge classes: two edges are in the same BCC iff they are equal or lie on a
  common simple cycle (paper, definition of BCCs as classes of that relation,
  in the preliminaries).  We enumerate every simple cycle and union the edges
  on it.  Parallel copies of an edge form a 2-cycle, so classes are computed
  on vertex pairs of the underlying simple graph.
* Articulation points: a vertex whose deletion increases the number of
  connected components (paper, Preliminaries).
"""
from __future__ import annotations

import itertools

import numpy as np


class _DSU:
    def __init__(self, n):
        self.p = list(range(n))

    def find(self, x):
        while self.p[x] != x:
            self.p[x] = self.p[self.p[x]]
            x = self.p[x]
        return x

    def union(self, a, b):
        a, b = self.find(a), self.find(b)
        if a != b:
            self.p[max(a, b)] = min(a, b)


def simple_cycles(n, pairs):
    """All simple cycles (length >= 3) of the simple graph with edge list
    ``pairs`` (each unordered pair once), each as a frozenset of pair indices.
    Each cycle is found from its smallest vertex, in both directions."""
    nbrs = [[] for _ in range(n)]
    for i, (a, b) in enumerate(pairs):
        nbrs[a].append((b, i))
        nbrs[b].append((a, i))
    out = set()

    def dfs(start, v, visited, used):
        for w, ei in nbrs[v]:
            if w == start and len(used) >= 2 and ei not in used:
                out.add(frozenset(used | {ei}))
            elif w > start and w not in visited:
                visited.add(w)
                dfs(start, w, visited, used | {ei})
                visited.remove(w)

    for s in range(n):
        dfs(s, s, {s}, frozenset())
    return out


def pair_classes(n, pairs, cycles=None):
    """Class representative (smallest pair index) for every pair."""
    if cycles is None:
        cycles = simple_cycles(n, pairs)
    d = _DSU(len(pairs))
    for c in cycles:
        c = sorted(c)
        for e in c[1:]:
            d.union(c[0], e)
    return [d.find(i) for i in range(len(pairs))]


def num_components(n, pairs, removed=None):
    d = _DSU(n)
    for a, b in pairs:
        if a != removed and b != removed:
            d.union(a, b)
    return len({d.find(v) for v in range(n) if v != removed})


def articulation_points(n, pairs):
    base = num_components(n, pairs)
    return np.array([1 if num_components(n, pairs, v) > base else 0 for v in range(n)], np.uint8)


def expected_from_csr(n, offsets, adj, cycles=None, pairs=None):
    """Canonical outputs (arc labels, AP flags, #BCC) for a CSR graph, from
    the definitions.  Arc label = smallest arc index whose edge is in the same
    class; -1 for self-loops."""
    offsets = np.asarray(offsets, np.int64)
    adj = np.asarray(adj, np.int64)
    src = np.repeat(np.arange(n), np.diff(offsets))
    if pairs is None:
        pairs = sorted({(min(u, v), max(u, v)) for u, v in zip(src.tolist(), adj.tolist()) if u != v})
    index = {p: i for i, p in enumerate(pairs)}
    cls = pair_classes(n, pairs, cycles)
    arc_cls = np.array(
        [cls[index[(min(u, v), max(u, v))]] if u != v else -1 for u, v in zip(src.tolist(), adj.tolist())],
        np.int64,
    )
    label = np.full(adj.shape[0], -1, np.int64)
    first_arc = {}
    for a, c in enumerate(arc_cls.tolist()):
        if c >= 0 and c not in first_arc:
            first_arc[c] = a
    for a, c in enumerate(arc_cls.tolist()):
        if c >= 0:
            label[a] = first_arc[c]
    ap = articulation_points(n, pairs)
    return label.astype(np.int32), ap, len(first_arc)


def complete_graph_cycles(n):
    """Pair list of K_n (lexicographic) and all its simple cycles as bitmasks
    over that list, for exhaustive enumeration of graphs on n vertices."""
    pairs = list(itertools.combinations(range(n), 2))
    cyc = simple_cycles(n, pairs)
    masks = np.array([sum(1 << i for i in c) for c in cyc], dtype=np.int64)
    return pairs, masks
