"""Seeded synthetic graph workloads (host side, shared by every consumer).

The generators live in ``graphgen.cpp`` (built into ``libgraphgen.so`` beside
this file).  They only draw random numbers and assemble symmetric CSR; no
biconnectivity arithmetic happens here, so the HIP path and the CPU oracle can
both take their inputs from this module without sharing any of the method.

Every CSR returned here is symmetric, with rows sorted ascending, no
self-loops and no repeated edges.  ``Csr.offsets`` is int64; ``Csr.offsets32()``
gives the int32 form when the arc count allows it.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from .. import build as _build

        _build.build_gen()
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, u64, f64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_int
    lib.gg_plain.restype = vp
    lib.gg_plain.argtypes = [u64, i64, i64, i64, i64, i64, i64, i64, i64]
    lib.gg_grid.restype = vp
    lib.gg_grid.argtypes = [u64, i64, i64, f64, i64, i64, i32]
    lib.gg_rmat.restype = vp
    lib.gg_rmat.argtypes = [u64, i32, i64, f64, f64, f64, i32]
    lib.gg_family.restype = vp
    lib.gg_family.argtypes = [u64, i32, i64, f64]
    lib.gg_mixed.restype = vp
    lib.gg_mixed.argtypes = [u64, i64, i64, i64, f64, f64]
    lib.gg_batch.restype = vp
    lib.gg_batch.argtypes = [u64, i64, i64, i64, f64, f64]
    lib.gg_from_edges.restype = vp
    lib.gg_from_edges.argtypes = [i64, i64, vp, vp]
    for name in ("gg_num_vertices", "gg_num_arcs", "gg_num_graphs", "gg_meta_len"):
        getattr(lib, name).restype = i64
        getattr(lib, name).argtypes = [vp]
    lib.gg_copy.restype = None
    lib.gg_copy.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.gg_free.restype = None
    lib.gg_free.argtypes = [vp]
    _lib = lib
    return lib


@dataclass
class Csr:
    """Symmetric CSR graph (optionally a disjoint union of several graphs)."""

    n: int
    offsets: np.ndarray  # int64 [n + 1]
    adj: np.ndarray  # int32 [num_arcs]
    vbegin: Optional[np.ndarray] = None  # int32 [G + 1] for unions
    meta: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int64))

    @property
    def num_arcs(self) -> int:
        return int(self.adj.shape[0])

    def offsets32(self) -> np.ndarray:
        if self.num_arcs >= 2**31:
            raise ValueError("arc count does not fit int32 offsets")
        return self.offsets.astype(np.int32)

    def degrees(self) -> np.ndarray:
        return np.diff(self.offsets)


def _take(h) -> Csr:
    lib = _load()
    try:
        n = lib.gg_num_vertices(h)
        a = lib.gg_num_arcs(h)
        g = lib.gg_num_graphs(h)
        ml = lib.gg_meta_len(h)
        off = np.empty(n + 1, np.int64)
        adj = np.empty(a, np.int32)
        vb = np.empty(g + 1, np.int32) if g > 0 else None
        meta = np.empty(ml, np.int64)
        lib.gg_copy(
            h,
            off.ctypes.data,
            None,
            adj.ctypes.data,
            vb.ctypes.data if vb is not None else None,
            meta.ctypes.data if ml else None,
        )
    finally:
        lib.gg_free(h)
    return Csr(int(n), off, adj, vb, meta)


def plain(seed=1, n_base=1 << 17, m_base=1 << 19, n_pendant=1 << 12, pmin=2, pmax=16,
          n_cycles=64, cmin=100, cmax=1000) -> Csr:
    """Uniform random base graph plus pendant trees and bridged cycles."""
    return _take(_load().gg_plain(seed, n_base, m_base, n_pendant, pmin, pmax, n_cycles, cmin, cmax))


def grid(seed=2, rows=4096, cols=4096, p=0.7, path_len=1 << 22, chord_block=1000, wrap=False) -> Csr:
    """Percolated lattice (open, or a torus with ``wrap``) plus a long chorded
    path hung off one corner."""
    return _take(_load().gg_grid(seed, rows, cols, p, path_len, chord_block, 1 if wrap else 0))


def rmat(seed=3, scale=25, edge_factor=16, a=0.57, b=0.19, c=0.19, permute=True) -> Csr:
    """R-MAT power-law graph, symmetrised, merged, ids permuted."""
    return _take(_load().gg_rmat(seed, scale, edge_factor, a, b, c, 1 if permute else 0))


FAMILIES = ("random", "lattice", "knn", "tree_back")


def family(name: str, n: int, param: float, seed=0) -> Csr:
    """One graph of a single family: random (param = mean degree), lattice
    (param = keep probability), knn (param = k), tree_back (param = fraction
    of extra ancestor edges)."""
    return _take(_load().gg_family(seed, FAMILIES.index(name), n, float(param)))


def mixed(seed: int, index: int, nmin: int, nmax: int, dmin: float, dmax: float) -> Csr:
    """Graph ``index`` of the mixed-family stream ``seed``."""
    return _take(_load().gg_mixed(seed, index, nmin, nmax, dmin, dmax))


def batch(seed=4, count=4096, nmin=64, nmax=1 << 16, dmin=4.0, dmax=16.0) -> Csr:
    """Disjoint union of ``count`` mixed-family graphs with vertex ranges."""
    return _take(_load().gg_batch(seed, count, nmin, nmax, dmin, dmax))


def from_edges(n: int, edges) -> Csr:
    """Symmetric merged CSR from an undirected edge list (pairs)."""
    e = np.asarray(edges, dtype=np.int32).reshape(-1, 2)
    u = np.ascontiguousarray(e[:, 0])
    v = np.ascontiguousarray(e[:, 1])
    return _take(_load().gg_from_edges(n, e.shape[0], u.ctypes.data, v.ctypes.data))


def multigraph_csr(n: int, edges) -> Csr:
    """Symmetric CSR that KEEPS repeated edges and self-loops (one arc per
    self-loop, two per ordinary edge), rows sorted.  For edge-case tests."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    src = np.concatenate([e[:, 0], e[e[:, 0] != e[:, 1], 1]])
    dst = np.concatenate([e[:, 1], e[e[:, 0] != e[:, 1], 0]])
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    off = np.zeros(n + 1, np.int64)
    np.add.at(off, src + 1, 1)
    off = np.cumsum(off)
    return Csr(n, off, dst.astype(np.int32))


def unite(graphs) -> Csr:
    """Disjoint union of CSR graphs with per-graph vertex ranges."""
    vb = np.zeros(len(graphs) + 1, np.int64)
    ab = np.zeros(len(graphs) + 1, np.int64)
    for i, g in enumerate(graphs):
        vb[i + 1] = vb[i] + g.n
        ab[i + 1] = ab[i] + g.num_arcs
    off = np.zeros(vb[-1] + 1, np.int64)
    adj = np.empty(ab[-1], np.int32)
    for i, g in enumerate(graphs):
        off[vb[i] : vb[i + 1] + 1] = g.offsets + ab[i]
        adj[ab[i] : ab[i + 1]] = g.adj + vb[i]
    return Csr(int(vb[-1]), off, adj, vb.astype(np.int32))


# Named workloads.  Full sizes are the benchmark configurations; "small"
# variants keep the same recipe at sizes a CPU test finishes in seconds.
def config(name: str) -> Csr:
    if name == "plain":
        return plain()
    if name == "plain_small":
        return plain(seed=11, n_base=1 << 12, m_base=1 << 14, n_pendant=64, n_cycles=8, cmin=10, cmax=60)
    if name == "grid":
        return grid()
    if name == "grid_small":
        return grid(seed=12, rows=128, cols=96, path_len=5000, chord_block=100)
    if name == "rmat":
        return rmat()
    if name == "rmat_small":
        return rmat(seed=13, scale=14)
    if name == "batch":
        return batch()
    if name == "batch_small":
        return batch(seed=14, count=64, nmin=16, nmax=2048)
    # circular grids of the paper's Table 1 shapes (SQR' and REC': 10^8
    # vertices, each edge kept with p = 0.6), and smaller ones of the same shape
    if name == "sqr_torus":
        return grid(seed=8, rows=10_000, cols=10_000, p=0.6, path_len=0, wrap=True)
    if name == "rec_torus":
        return grid(seed=9, rows=1_000, cols=100_000, p=0.6, path_len=0, wrap=True)
    if name == "sqr_torus_2000":
        return grid(seed=8, rows=2_000, cols=2_000, p=0.6, path_len=0, wrap=True)
    if name == "rec_torus_400":
        return grid(seed=9, rows=400, cols=10_000, p=0.6, path_len=0, wrap=True)
    if name.startswith("knn"):  # "knn<k>": 2^22 points in the unit square, k nearest neighbours
        return family("knn", 1 << 22, int(name[3:]), seed=6)
    raise KeyError(name)
