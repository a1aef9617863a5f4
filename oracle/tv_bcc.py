"""Tarjan-Vishkin BCC with an explicit skeleton -- TEST INFRASTRUCTURE ONLY.

A second CPU solver, independent of both the Hopcroft-Tarjan oracle and the
HIP path, used to cross-check them on medium graphs and to measure how large
the Tarjan-Vishkin skeleton is (the paper's space argument).  Only tests/
and the benchmark's reporting may import it.

Steps (paper: Section "The Tarjan-Vishkin Algorithm" and the appendix on
Tarjan-Vishkin, which defines the skeleton G' = (E, E')):
  1. an arbitrary spanning forest T -- here a breadth-first forest from the
     smallest unvisited vertex (any spanning forest works);
  2. root it and number it in preorder: first[v]; last[v] = first[v] + |T_v| - 1;
  3. w1[u] = min({first[u]} U {first[u'] : u-u' non-tree}), w2 likewise with
     max; low[v] / high[v] = min / max of w1 / w2 over T_v;
  4. G' has one vertex per edge of G, and e1 ~ e2 when
       (a) e1 = (u, p(u)), e2 = (u, v) non-tree with first[v] < first[u];
       (b) e1 = (u, p(u)), e2 = (v, p(v)) and u-v is a cross edge;
       (c) e1 = (u, v) with v = p(u) not a root, e2 = (v, p(v)), and some
           non-tree edge leaves T_u for a vertex outside T_v
           (low[u] < first[v] or high[u] > last[v]);
  5. connected components of G' are the BCCs of G.
Output follows the oracle's conventions: arc label = smallest arc index of
the BCC, -1 for self-loops.  scipy's graph routines (BFS order, connected
components) serve as library primitives.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import breadth_first_order, connected_components


def _pair_arcs(n, off, adj):
    """Undirected edge id for every arc (both arcs of an edge share it; the
    k-th copy u->w in row u pairs with the k-th copy w->u in row w); -1 for
    self-loops.  Returns (edge_of_arc, edge_u, edge_v)."""
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(off))
    dst = adj.astype(np.int64)
    A = len(dst)
    lo, hi = np.minimum(src, dst), np.maximum(src, dst)
    # group both directions of each unordered pair, rank copies within a row
    key_dir = np.lexsort((np.arange(A), dst, src))  # arcs sorted by (src, dst, index)
    rank = np.empty(A, np.int64)
    s_sorted, d_sorted = src[key_dir], dst[key_dir]
    start = np.r_[True, (s_sorted[1:] != s_sorted[:-1]) | (d_sorted[1:] != d_sorted[:-1])]
    grp = np.cumsum(start) - 1
    first_in_grp = np.flatnonzero(start)
    rank[key_dir] = np.arange(A) - first_in_grp[grp]
    # edge key = (lo, hi, rank); the two arcs of an edge share it
    edge_of_arc = -np.ones(A, np.int64)
    nl = src != dst
    keys = np.stack([lo[nl], hi[nl], rank[nl]], 1)
    uniq, inv = np.unique(keys, axis=0, return_inverse=True)
    edge_of_arc[np.flatnonzero(nl)] = inv.reshape(-1)
    return edge_of_arc, uniq[:, 0], uniq[:, 1]


def _spanning_forest(n, eu, ev):
    """Breadth-first forest rooted at each component's smallest vertex (one
    BFS from a virtual source joined to those roots): parent[v] (-1 for
    roots), preorder first[v], last[v], and the preorder itself."""
    m = len(eu)
    g = sp.csr_matrix((np.ones(2 * m), (np.r_[eu, ev], np.r_[ev, eu])), shape=(n, n))
    ncomp, comp = connected_components(g, directed=False)
    roots = np.full(ncomp, n, np.int64)
    np.minimum.at(roots, comp, np.arange(n))
    src = n  # virtual source
    gx = sp.csr_matrix((np.ones(2 * m + 2 * ncomp), (np.r_[eu, ev, np.full(ncomp, src), roots],
                                                        np.r_[ev, eu, roots, np.full(ncomp, src)])),
                       shape=(n + 1, n + 1))
    _, pred = breadth_first_order(gx, src, directed=False, return_predecessors=True)
    parent = pred[:n].astype(np.int64)
    parent[parent == src] = -1
    # preorder: depth-first order of the forest from the same virtual source
    child = np.arange(n)
    par = np.where(parent >= 0, parent, src)
    tree = sp.csr_matrix((np.ones(n), (par, child)), shape=(n + 1, n + 1))
    order = sp.csgraph.depth_first_order(tree, src, directed=True, return_predecessors=False)[1:]
    first = np.empty(n, np.int64)
    first[order] = np.arange(n)
    size = np.ones(n, np.int64)
    par_l = parent.tolist()
    size_l = size.tolist()
    for v in reversed(order.tolist()):  # children before parents
        p = par_l[v]
        if p >= 0:
            size_l[p] += size_l[v]
    last = first + np.asarray(size_l, np.int64) - 1
    return parent, first, last, order.tolist()


def tv_bcc(offsets, adj, return_skeleton_size=False):
    off = np.asarray(offsets, np.int64)
    a = np.asarray(adj, np.int64)
    n = len(off) - 1
    A = len(a)
    edge_of_arc, eu, ev = _pair_arcs(n, off, a)
    m = len(eu)
    parent, first, last, post = _spanning_forest(n, eu, ev)
    # which undirected edges are tree edges: the first copy of (v, parent[v])
    is_tree = np.zeros(m, bool)
    tree_edge_of = -np.ones(n, np.int64)  # tree edge (v, p(v)) by child v
    order = np.lexsort((np.arange(m), ev, eu))
    keys = eu[order] * n + ev[order]
    ch = np.flatnonzero(parent >= 0)
    ck = np.minimum(ch, parent[ch]) * n + np.maximum(ch, parent[ch])
    e = order[np.searchsorted(keys, ck)]
    tree_edge_of[ch] = e
    is_tree[e] = True
    # w1 / w2 over non-tree neighbours, then subtree min / max
    w1 = first.copy()
    w2 = first.copy()
    nt = ~is_tree
    for x, y in ((eu[nt], ev[nt]), (ev[nt], eu[nt])):
        np.minimum.at(w1, x, first[y])
        np.maximum.at(w2, x, first[y])
    low, high = w1.tolist(), w2.tolist()
    par_l = parent.tolist()
    for v in reversed(post):
        p = par_l[v]
        if p >= 0:
            if low[v] < low[p]:
                low[p] = low[v]
            if high[v] > high[p]:
                high[p] = high[v]
    low, high = np.asarray(low, np.int64), np.asarray(high, np.int64)
    # skeleton edges
    E1, E2 = [], []
    ntu, ntv = eu[nt], ev[nt]
    nte = np.flatnonzero(nt)
    # (a): the later endpoint's tree edge ~ the non-tree edge
    later = np.where(first[ntu] > first[ntv], ntu, ntv)
    ok = parent[later] >= 0
    E1.append(tree_edge_of[later[ok]])
    E2.append(nte[ok])
    # (b): cross edges join the two tree edges of their endpoints
    anc_uv = (first[ntu] <= first[ntv]) & (first[ntv] <= last[ntu])
    anc_vu = (first[ntv] <= first[ntu]) & (first[ntu] <= last[ntv])
    cross = ~anc_uv & ~anc_vu & (parent[ntu] >= 0) & (parent[ntv] >= 0)
    E1.append(tree_edge_of[ntu[cross]])
    E2.append(tree_edge_of[ntv[cross]])
    # (c): tree edge (u, v = p(u)) ~ (v, p(v)) when T_u escapes T_v
    u = np.flatnonzero(parent >= 0)
    v = parent[u]
    ok = parent[v] >= 0
    u, v = u[ok], v[ok]
    esc = (low[u] < first[v]) | (high[u] > last[v])
    E1.append(tree_edge_of[u[esc]])
    E2.append(tree_edge_of[v[esc]])
    e1 = np.concatenate(E1)
    e2 = np.concatenate(E2)
    skel = sp.csr_matrix((np.ones(len(e1)), (e1, e2)), shape=(m, m))
    _, comp = connected_components(skel, directed=False)
    # canonical labels: smallest arc index per class
    label = -np.ones(A, np.int64)
    has = edge_of_arc >= 0
    cls = comp[edge_of_arc[has]]
    best = np.full(comp.max() + 1 if m else 0, np.iinfo(np.int64).max)
    np.minimum.at(best, cls, np.flatnonzero(has))
    label[has] = best[cls]
    num_bcc = len(np.unique(cls)) if m else 0
    # articulation points: vertices incident to two or more classes
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(off))
    pairs = np.unique(np.stack([src[has], cls], 1), axis=0) if m else np.zeros((0, 2), np.int64)
    ap = (np.bincount(pairs[:, 0], minlength=n) >= 2).astype(np.uint8)
    out = (label.astype(np.int32), ap, num_bcc)
    if return_skeleton_size:
        return out + ({"skeleton_vertices": m, "skeleton_edges": int(len(e1))},)
    return out
