"""FAST-BCC biconnected components on one MI355X.

The compute path is ``libfastbcc.so`` (hand-written HIP for gfx950, C ABI in
``include/fastbcc.h``); this package only marshals torch tensors into it.
"""
from .api import (  # noqa: F401
    BccResult,
    alloc_workspace,
    batch_rebase,
    bc_labeling,
    check_batched,
    read_device_status,
    solve,
    solve_batched,
    solve_noalloc,
    solve_small,
    solve_traced,
    vertex_labels,
    workspace_size,
)

__all__ = ["BccResult", "alloc_workspace", "batch_rebase", "bc_labeling", "check_batched", "read_device_status", "solve", "solve_batched", "solve_noalloc", "solve_small", "solve_traced", "vertex_labels",
           "workspace_size"]
