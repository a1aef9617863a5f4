"""The allocation-free entry point (fastbcc_solve_noalloc, static per-GPU
scratch) against the workspace entry point (fastbcc_solve) through the C
ABI: bit-exact labels, articulation points and BCC counts on consecutive
calls, the later ones on smaller graphs (the scratch keeps the earlier
call's contents), and the refusal of a graph too large for the scratch."""
import ctypes
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2301_01356_amd import _native as N
from paper_2301_01356_amd import gen

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def run(entry, g, flags):
    """One solve through the C ABI; returns host (labels, AP flags, #BCC)."""
    lib = N.lib()
    off = torch.from_numpy(g.offsets32()).to(DEV)
    adj = torch.from_numpy(g.adj).to(DEV)
    lab = torch.full((g.num_arcs,), -7, dtype=torch.int32, device=DEV)
    ap = torch.full((g.n,), 9, dtype=torch.uint8, device=DEV)
    nb = torch.full((1,), -7, dtype=torch.int64, device=DEV)
    st = torch.cuda.current_stream().cuda_stream
    args = (g.n, g.num_arcs, off.data_ptr(), adj.data_ptr() if g.num_arcs else None,
            lab.data_ptr() if g.num_arcs else None, ap.data_ptr() if g.n else None, nb.data_ptr())
    if entry == "noalloc":
        rc = lib.fastbcc_solve_noalloc(*args, flags, st)
        ws = None
    else:
        need = N.workspace_size(g.n, g.num_arcs, 1)
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=DEV)
        rc = lib.fastbcc_solve(*args, ws.data_ptr(), ws.numel(), flags, st)
    assert rc == N.OK, f"{entry}: status {rc}"
    if ws is not None:
        out = ctypes.c_int32(-1)
        assert lib.fastbcc_read_device_status(ws.data_ptr(), st, ctypes.byref(out)) == N.OK
        assert out.value == 0
    torch.cuda.synchronize()
    return lab.cpu().numpy(), ap.cpu().numpy(), int(nb.item())


def same(a, b):
    return np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]


PROMISED = N.FLAG_SORTED_ROWS | N.FLAG_NO_SELF_LOOPS | N.tune_flags(sampled_tags=True, free_first_round=True)


def test_noalloc_equals_workspace_solve_on_consecutive_calls():
    # the full plain workload (39 MiB of workspace) first, then smaller graphs
    cases = [("plain", gen.config("plain"), PROMISED), ("plain_small", gen.config("plain_small"), 0),
             ("rmat_small", gen.config("rmat_small"), PROMISED), ("grid_small", gen.config("grid_small"), 0),
             ("path3", gen.from_edges(3, [(0, 1), (1, 2)]), 0)]
    for name, g, flags in cases:
        assert N.workspace_size(g.n, g.num_arcs, 1) <= N.NOALLOC_SCRATCH_BYTES
        note(f"noalloc {name} n={g.n} arcs={g.num_arcs} flags={flags:#x}")
        got = run("noalloc", g, flags)
        note(f"workspace solve {name}")
        want = run("workspace", g, flags)
        assert same(got, want), f"{name}: the allocation-free solve differs from the workspace solve"
        lab, ap, nb, _, _ = oracle.ht_bcc(g.offsets, g.adj)
        assert same(got, (lab, ap, nb)), f"{name}: differs from the oracle"


def test_noalloc_refuses_graphs_beyond_the_scratch():
    lib = N.lib()
    n, A = 1 << 22, 1 << 24  # a workspace of about 1 GB
    assert N.workspace_size(n, A, 1) > N.NOALLOC_SCRATCH_BYTES
    note("noalloc refusal (no launch)")
    rc = lib.fastbcc_solve_noalloc(n, A, None, None, None, None, None, 0, None)
    assert rc == N.ERR_SCRATCH_TOO_SMALL
    assert "scratch" in lib.fastbcc_status_string(rc).decode()
