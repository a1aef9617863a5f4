"""Torch-facing wrappers over the C ABI (marshalling only).

PyTorch provides device memory and streams; every step of the solve runs in
the HIP kernels of ``libfastbcc.so``.  Names follow the C ABI:

* ``workspace_size(n, num_arcs, num_graphs=1)``
* ``solve(offsets, adj, ...)``          -- one graph, int32 or int64 offsets
* ``solve_batched(vbegin, offsets, adj, ...)`` -- many graphs, one launch sequence
* ``read_device_status(workspace)``
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import torch

from . import _native as N


@dataclass
class BccResult:
    edge_label: torch.Tensor  # int32 [num_arcs]: smallest arc id of the arc's BCC, -1 for self-loops
    is_ap: torch.Tensor  # uint8 [n]: articulation-point flags
    num_bcc: torch.Tensor  # int64 [num_graphs]


def _dev_ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _check_tensor(t: torch.Tensor, name: str, dtypes, numel=None, device=None):
    """Refuse anything the kernels cannot read as a plain device array: host or
    foreign-device tensors, wrong dtypes, strided views, wrong sizes."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must live on a GPU (got {t.device})")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, the graph on {device}")
    if t.dtype not in dtypes:
        raise TypeError(f"{name} has dtype {t.dtype}, expected one of {dtypes}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")


def _check_workspace(ws: torch.Tensor, n: int, num_arcs: int, num_graphs: int, device) -> None:
    """The workspace must be a contiguous uint8 buffer on the graph's device,
    large enough (the library checks size and alignment too, but cannot tell
    a host pointer from a device one)."""
    _check_tensor(ws, "workspace", (torch.uint8,), device=device)
    need = workspace_size(n, num_arcs, num_graphs)
    if ws.numel() < need:
        raise ValueError(f"workspace has {ws.numel()} bytes, the solve needs {need}")


def _check_result(out: "BccResult", n: int, A: int, G: int, device) -> None:
    _check_tensor(out.edge_label, "edge_label", (torch.int32,), A, device)
    _check_tensor(out.is_ap, "is_ap", (torch.uint8,), n, device)
    _check_tensor(out.num_bcc, "num_bcc", (torch.int64,), G, device)


def workspace_size(n: int, num_arcs: int, num_graphs: int = 1) -> int:
    return N.workspace_size(n, num_arcs, num_graphs)


def alloc_workspace(n: int, num_arcs: int, num_graphs: int = 1, device=None) -> torch.Tensor:
    """Caller-owned workspace (torch allocation, 256-byte aligned)."""
    nbytes = workspace_size(n, num_arcs, num_graphs)
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device or "cuda")


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def solve(
    offsets: torch.Tensor,
    adj: torch.Tensor,
    *,
    out: Optional[BccResult] = None,
    workspace: Optional[torch.Tensor] = None,
    flags: int = 0,
    stream=None,
) -> BccResult:
    """BCCs of one graph given as symmetric CSR on the GPU (asynchronous on ``stream``)."""
    _check_tensor(offsets, "offsets", (torch.int32, torch.int64))
    n = offsets.numel() - 1
    if n < 0:
        raise ValueError("offsets needs n + 1 >= 1 entries")
    dev = offsets.device
    _check_tensor(adj, "adj", (torch.int32,), device=dev)
    A = adj.numel()
    if out is None:
        out = BccResult(
            torch.empty(A, dtype=torch.int32, device=dev),
            torch.empty(n, dtype=torch.uint8, device=dev),
            torch.empty(1, dtype=torch.int64, device=dev),
        )
    _check_result(out, n, A, 1, dev)
    if workspace is None:
        workspace = alloc_workspace(n, A, 1, dev)
    _check_workspace(workspace, n, A, 1, dev)
    fn = N.lib().fastbcc_solve if offsets.dtype == torch.int32 else N.lib().fastbcc_solve_off64
    with torch.cuda.device(dev):
        st = fn(
            n,
            A,
            offsets.data_ptr(),
            _dev_ptr(adj) if A else None,
            _dev_ptr(out.edge_label) if A else None,
            _dev_ptr(out.is_ap) if n else None,
            out.num_bcc.data_ptr(),
            workspace.data_ptr(),
            workspace.numel(),
            flags,
            _stream_handle(stream),
        )
    N.check(st, "fastbcc_solve")
    return out


def solve_noalloc(
    offsets: torch.Tensor,
    adj: torch.Tensor,
    *,
    out: BccResult,
    flags: int = 0,
    stream=None,
) -> BccResult:
    """``solve`` in the library's static per-GPU scratch instead of a
    workspace: the call allocates nothing (``out`` is the caller's).  Graphs
    whose workspace would exceed ``NOALLOC_SCRATCH_BYTES`` are refused; calls
    that overlap on one GPU race on the shared scratch."""
    _check_tensor(offsets, "offsets", (torch.int32,))
    n = offsets.numel() - 1
    if n < 0:
        raise ValueError("offsets needs n + 1 >= 1 entries")
    dev = offsets.device
    _check_tensor(adj, "adj", (torch.int32,), device=dev)
    A = adj.numel()
    _check_result(out, n, A, 1, dev)
    with torch.cuda.device(dev):
        st = N.lib().fastbcc_solve_noalloc(
            n,
            A,
            offsets.data_ptr(),
            _dev_ptr(adj) if A else None,
            _dev_ptr(out.edge_label) if A else None,
            _dev_ptr(out.is_ap) if n else None,
            out.num_bcc.data_ptr(),
            flags,
            _stream_handle(stream),
        )
    N.check(st, "fastbcc_solve_noalloc")
    return out


def solve_batched(
    vbegin: torch.Tensor,
    offsets: torch.Tensor,
    adj: torch.Tensor,
    *,
    out: Optional[BccResult] = None,
    workspace: Optional[torch.Tensor] = None,
    flags: int = 0,
    stream=None,
) -> BccResult:
    """BCCs of many graphs concatenated as one CSR (graph g owns vertices
    vbegin[g]..vbegin[g+1]); labels are graph-local, num_bcc is per graph."""
    _check_tensor(offsets, "offsets", (torch.int32,))
    dev = offsets.device
    _check_tensor(vbegin, "vbegin", (torch.int32,), device=dev)
    _check_tensor(adj, "adj", (torch.int32,), device=dev)
    G = vbegin.numel() - 1
    if G < 1:
        raise ValueError("vbegin needs at least 2 entries")
    n = offsets.numel() - 1
    if n < 0:
        raise ValueError("offsets needs n + 1 >= 1 entries")
    A = adj.numel()
    if out is None:
        out = BccResult(
            torch.empty(A, dtype=torch.int32, device=dev),
            torch.empty(n, dtype=torch.uint8, device=dev),
            torch.empty(G, dtype=torch.int64, device=dev),
        )
    _check_result(out, n, A, G, dev)
    if workspace is None:
        workspace = alloc_workspace(n, A, G, dev)
    _check_workspace(workspace, n, A, G, dev)
    with torch.cuda.device(dev):
        st = N.lib().fastbcc_solve_batched(
            G,
            vbegin.data_ptr(),
            n,
            A,
            offsets.data_ptr(),
            _dev_ptr(adj) if A else None,
            _dev_ptr(out.edge_label) if A else None,
            _dev_ptr(out.is_ap) if n else None,
            out.num_bcc.data_ptr(),
            workspace.data_ptr(),
            workspace.numel(),
            flags,
            _stream_handle(stream),
        )
    N.check(st, "fastbcc_solve_batched")
    return out


def solve_small(
    vbegin: torch.Tensor,
    offsets: torch.Tensor,
    adj: torch.Tensor,
    *,
    packs: Optional[torch.Tensor] = None,
    out: Optional[BccResult] = None,
    flags: int = 0,
    stream=None,
) -> BccResult:
    """As ``solve_batched`` for small graphs, by the fused kernels (one
    workgroup per pack of consecutive graphs, all state in LDS, no
    workspace).  ``packs``: int32 pack starts (graph indices, from 0 to G),
    or None for one graph per pack.  A pack above ``SMALL_MAX_VERTICES``
    vertices or graphs gets num_bcc = -1 for its graphs and no labels."""
    _check_tensor(offsets, "offsets", (torch.int32,))
    dev = offsets.device
    _check_tensor(vbegin, "vbegin", (torch.int32,), device=dev)
    _check_tensor(adj, "adj", (torch.int32,), device=dev)
    G = vbegin.numel() - 1
    if G < 1:
        raise ValueError("vbegin needs at least 2 entries")
    P = 0
    if packs is not None:
        _check_tensor(packs, "packs", (torch.int32,), device=dev)
        P = packs.numel() - 1
        if P < 1:
            raise ValueError("packs needs at least 2 entries")
    n = offsets.numel() - 1
    if n < 0:
        raise ValueError("offsets needs n + 1 >= 1 entries")
    A = adj.numel()
    if out is None:
        out = BccResult(
            torch.empty(A, dtype=torch.int32, device=dev),
            torch.empty(n, dtype=torch.uint8, device=dev),
            torch.empty(G, dtype=torch.int64, device=dev),
        )
    _check_result(out, n, A, G, dev)
    with torch.cuda.device(dev):
        st = N.lib().fastbcc_solve_small(
            G,
            vbegin.data_ptr(),
            P,
            packs.data_ptr() if packs is not None else None,
            n,
            A,
            offsets.data_ptr(),
            _dev_ptr(adj) if A else None,
            _dev_ptr(out.edge_label) if A else None,
            _dev_ptr(out.is_ap) if n else None,
            out.num_bcc.data_ptr(),
            flags,
            _stream_handle(stream),
        )
    N.check(st, "fastbcc_solve_small")
    return out


def solve_traced(
    offsets: torch.Tensor,
    adj: torch.Tensor,
    trace: "N.Trace",
    *,
    vbegin: Optional[torch.Tensor] = None,
    out: Optional[BccResult] = None,
    workspace: Optional[torch.Tensor] = None,
    flags: int = 0,
    stream=None,
) -> BccResult:
    """``solve``/``solve_batched`` with an event pair around every kernel."""
    _check_tensor(offsets, "offsets", (torch.int32, torch.int64))
    dev = offsets.device
    _check_tensor(adj, "adj", (torch.int32,), device=dev)
    n = offsets.numel() - 1
    if n < 0:
        raise ValueError("offsets needs n + 1 >= 1 entries")
    A = adj.numel()
    G = 1
    if vbegin is not None:
        _check_tensor(vbegin, "vbegin", (torch.int32,), device=dev)
        G = vbegin.numel() - 1
        if G < 1:
            raise ValueError("vbegin needs at least 2 entries")
        if offsets.dtype != torch.int32:
            raise TypeError("batched solves take int32 offsets")
    if out is None:
        out = BccResult(
            torch.empty(A, dtype=torch.int32, device=dev),
            torch.empty(n, dtype=torch.uint8, device=dev),
            torch.empty(G, dtype=torch.int64, device=dev),
        )
    _check_result(out, n, A, G, dev)
    if workspace is None:
        workspace = alloc_workspace(n, A, G, dev)
    _check_workspace(workspace, n, A, G, dev)
    with torch.cuda.device(dev):
        st = N.lib().fastbcc_solve_traced(
            G,
            _dev_ptr(vbegin),
            n,
            A,
            offsets.data_ptr(),
            32 if offsets.dtype == torch.int32 else 64,
            _dev_ptr(adj) if A else None,
            _dev_ptr(out.edge_label) if A else None,
            _dev_ptr(out.is_ap) if n else None,
            out.num_bcc.data_ptr(),
            workspace.data_ptr(),
            workspace.numel(),
            flags,
            _stream_handle(stream),
            trace.h,
        )
    N.check(st, "fastbcc_solve_traced")
    return out


def vertex_labels(workspace: torch.Tensor, n: int, num_arcs: int, vbegin: Optional[torch.Tensor] = None,
                  stream=None):
    """BC-labeling of the last solve on ``workspace``: (home int32[n], home_head
    int32[n]) -- each vertex's home BCC (canonical id) and that BCC's head;
    -1 for spanning-tree roots."""
    _check_tensor(workspace, "workspace", (torch.uint8,))
    dev = workspace.device
    G = 1
    if vbegin is not None:
        _check_tensor(vbegin, "vbegin", (torch.int32,), device=dev)
        G = vbegin.numel() - 1
        if G < 1:
            raise ValueError("vbegin needs at least 2 entries")
    _check_workspace(workspace, n, num_arcs, G, dev)
    home = torch.empty(n, dtype=torch.int32, device=dev)
    head = torch.empty(n, dtype=torch.int32, device=dev)
    with torch.cuda.device(dev):
        st = N.lib().fastbcc_vertex_labels(n, num_arcs, G, _dev_ptr(vbegin), workspace.data_ptr(), workspace.numel(),
                                           home.data_ptr() if n else None, head.data_ptr() if n else None,
                                           _stream_handle(stream))
    N.check(st, "fastbcc_vertex_labels")
    return home, head


def greedy_packs(sizes, capacity: int = N.SMALL_MAX_VERTICES) -> list:
    """Pack starts for ``solve_small``: consecutive graphs are added to a
    pack while its vertex count stays within ``capacity`` (a graph above it
    forms a pack of its own) and its graph count within the fused kernels'
    limit."""
    starts, total, count = [0], 0, 0
    for i, v in enumerate(sizes):
        v = int(v)
        if count and (total + v > capacity or count >= N.SMALL_MAX_VERTICES):
            starts.append(i)
            total = count = 0
        total += v
        count += 1
    if count:
        starts.append(len(sizes))
    return starts


def batch_rebase(offsets: torch.Tensor, adj: torch.Tensor, vbegin: torch.Tensor, abegin: torch.Tensor,
                 stream=None) -> None:
    """Make the graph-local ids and row starts of a freshly copied batch
    global, in place (graph g: vertices vbegin[g].., arcs abegin[g]..)."""
    _check_tensor(offsets, "offsets", (torch.int32,))
    dev = offsets.device
    _check_tensor(adj, "adj", (torch.int32,), device=dev)
    _check_tensor(vbegin, "vbegin", (torch.int32,), device=dev)
    _check_tensor(abegin, "abegin", (torch.int32,), vbegin.numel(), dev)
    G = vbegin.numel() - 1
    if G < 1:
        raise ValueError("vbegin needs at least 2 entries")
    n, A = offsets.numel() - 1, adj.numel()
    with torch.cuda.device(dev):
        st = N.lib().fastbcc_batch_rebase(G, vbegin.data_ptr(), abegin.data_ptr(), n, A, offsets.data_ptr(),
                                          _dev_ptr(adj) if A else None, _stream_handle(stream))
    N.check(st, "fastbcc_batch_rebase")


def check_batched(offsets: torch.Tensor, adj: torch.Tensor, vbegin: Optional[torch.Tensor] = None, *,
                  flags: int = 0, repair: bool = False, out: Optional[torch.Tensor] = None,
                  stream=None) -> torch.Tensor:
    """Per-graph input check of a batch on the device (int32 status per
    graph, 0 = passed); ``repair`` rewrites failed graphs in place into valid
    ones so that a batched solve can follow at once."""
    _check_tensor(offsets, "offsets", (torch.int32,))
    dev = offsets.device
    _check_tensor(adj, "adj", (torch.int32,), device=dev)
    n, A = offsets.numel() - 1, adj.numel()
    G = 1
    if vbegin is not None:
        _check_tensor(vbegin, "vbegin", (torch.int32,), device=dev)
        G = vbegin.numel() - 1
        if G < 1:
            raise ValueError("vbegin needs at least 2 entries")
    if out is None:
        out = torch.empty(G, dtype=torch.int32, device=dev)
    _check_tensor(out, "status", (torch.int32,), G, dev)
    f = flags | (N.FLAG_REPAIR if repair else 0)
    with torch.cuda.device(dev):
        st = N.lib().fastbcc_check_batched(G, _dev_ptr(vbegin), n, A, offsets.data_ptr(), _dev_ptr(adj) if A else None,
                                           f, out.data_ptr(), _stream_handle(stream))
    N.check(st, "fastbcc_check_batched")
    return out


@dataclass
class BcLabeling:
    label: torch.Tensor  # int32 [n]: l[v], the vertex representing v's label (-1: tree root)
    parent: torch.Tensor  # int32 [n]: spanning-forest parent (-1: root)
    cut_parent: torch.Tensor  # int32 [n]: block-cut tree parent BCC of an articulation point (-1 otherwise)
    is_bridge: torch.Tensor  # uint8 [num_arcs]: arc of a one-edge BCC


def bc_labeling(workspace: torch.Tensor, offsets: torch.Tensor, adj: torch.Tensor, result: BccResult,
                vbegin: Optional[torch.Tensor] = None, flags: int = 0, stream=None) -> BcLabeling:
    """Labels l[], spanning-forest parents, block-cut tree parents of the
    articulation points and bridge arcs of the last solve on ``workspace``
    (``result`` is that solve's output)."""
    _check_tensor(offsets, "offsets", (torch.int32, torch.int64))
    dev = offsets.device
    _check_tensor(adj, "adj", (torch.int32,), device=dev)
    n, A = offsets.numel() - 1, adj.numel()
    G = 1
    if vbegin is not None:
        _check_tensor(vbegin, "vbegin", (torch.int32,), device=dev)
        G = vbegin.numel() - 1
    _check_result(result, n, A, G, dev)
    _check_workspace(workspace, n, A, G, dev)
    out = BcLabeling(torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.int32, device=dev),
                     torch.empty(n, dtype=torch.int32, device=dev), torch.empty(A, dtype=torch.uint8, device=dev))
    with torch.cuda.device(dev):
        st = N.lib().fastbcc_bc_labeling(
            n, A, G, _dev_ptr(vbegin), offsets.data_ptr(), 32 if offsets.dtype == torch.int32 else 64,
            _dev_ptr(adj) if A else None, _dev_ptr(result.edge_label) if A else None,
            _dev_ptr(result.is_ap) if n else None, workspace.data_ptr(), workspace.numel(), flags,
            out.label.data_ptr() if n else None, out.parent.data_ptr() if n else None,
            out.cut_parent.data_ptr() if n else None, out.is_bridge.data_ptr() if A else None,
            _stream_handle(stream))
    N.check(st, "fastbcc_bc_labeling")
    return out


def read_device_status(workspace: torch.Tensor, stream=None) -> int:
    """Synchronise ``stream`` and return the status word the last solve on
    ``workspace`` left (0 = no device-side check fired)."""
    import ctypes

    _check_tensor(workspace, "workspace", (torch.uint8,))
    out = ctypes.c_int32(0)
    N.check(N.lib().fastbcc_read_device_status(workspace.data_ptr(), _stream_handle(stream), ctypes.byref(out)))
    return int(out.value)
