"""Host-side checks of the C ABI (no GPU needed: nothing here launches work)."""
import ctypes
import os
import re

import pytest

from paper_2301_01356_amd import _native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fastbcc.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"FASTBCC_API\s+[\w\s\*]+?\b(fastbcc_\w+)\s*\(", text)))


def test_header_declares_the_bound_entry_points():
    assert declared_functions() == sorted(N.EXPORTED)


def test_library_loads_and_exports_every_declared_symbol():
    lib = N.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert lib.fastbcc_version().decode().count(".") == 2


def test_no_other_symbols_exported():
    import subprocess

    out = subprocess.run(["nm", "-D", "--defined-only", N.LIB_PATH], capture_output=True, text=True, check=True).stdout
    text_syms = sorted(l.split()[-1] for l in out.splitlines() if " T " in l)
    assert text_syms == sorted(N.EXPORTED)


def test_workspace_size_is_linear_in_n():
    a = N.workspace_size(1 << 16, 1 << 20)
    b = N.workspace_size(1 << 17, 1 << 20)
    c = N.workspace_size(1 << 17, 1 << 24)
    assert 0 < a < b
    # arcs only add bookkeeping: two int32 tile-row arrays (one entry per 256
    # arcs), 32 hub counters per possible hub (one hub per 4096 arcs) and one
    # descendant bit per arc
    assert c - b <= ((1 << 24) - (1 << 20)) // 4 + 4096
    # the O(n) part: well under 256 bytes per vertex
    assert b / (1 << 17) < 256


def test_workspace_size_rejects_bad_arguments():
    lib = N.lib()
    out = ctypes.c_size_t(0)
    assert lib.fastbcc_workspace_size(-1, 0, 1, ctypes.byref(out)) == N.ERR_INVALID_ARGUMENT
    assert lib.fastbcc_workspace_size(1 << 30, 0, 1, ctypes.byref(out)) == N.ERR_TOO_LARGE
    assert lib.fastbcc_workspace_size(10, 1 << 31, 1, ctypes.byref(out)) == N.ERR_TOO_LARGE
    assert lib.fastbcc_workspace_size(10, 10, 1, None) == N.ERR_INVALID_ARGUMENT


def _solve(n, arcs, ws, ws_bytes, flags=0, off=1):
    # pointers are never dereferenced on these error paths
    return N.lib().fastbcc_solve(n, arcs, off, 1, 1, None, None, ws, ws_bytes, flags, None)


def test_solve_argument_errors_are_synchronous():
    need = N.workspace_size(100, 400)
    assert _solve(100, 400, None, need) == N.ERR_WORKSPACE_TOO_SMALL
    assert _solve(100, 400, 256, need - 1) == N.ERR_WORKSPACE_TOO_SMALL
    assert _solve(100, 400, 256 + 4, need) == N.ERR_INVALID_ARGUMENT  # misaligned workspace
    assert _solve(-5, 400, 256, need) == N.ERR_INVALID_ARGUMENT
    assert _solve(1 << 30, 400, 256, 1 << 40) == N.ERR_TOO_LARGE
    assert _solve(100, 400, 256, need, flags=2 << N.TUNE_RULER_SHIFT) == N.ERR_INVALID_ARGUMENT
    assert _solve(100, 400, 256, need, flags=1 << N.TUNE_TILE_SHIFT) == N.ERR_INVALID_ARGUMENT
    assert _solve(100, 400, 256, need, off=0) == N.ERR_INVALID_ARGUMENT
    lib = N.lib()
    assert lib.fastbcc_solve_batched(0, 1, 10, 10, 1, 1, 1, None, None, 256, need, 0, None) == N.ERR_INVALID_ARGUMENT
    assert lib.fastbcc_solve_batched(2, None, 10, 10, 1, 1, 1, None, None, 256, need, 0, None) == N.ERR_INVALID_ARGUMENT
    st = ctypes.c_int32(0)
    assert lib.fastbcc_read_device_status(None, None, ctypes.byref(st)) == N.ERR_INVALID_ARGUMENT


def test_solve_small_argument_errors_are_synchronous():
    """Refused before anything touches the GPU (pointers are never read)."""
    f = N.lib().fastbcc_solve_small
    # graphs, vbegin, packs, pack_begin, n, arcs, offsets, adj, label, ap, nbcc, flags, stream
    assert f(0, 256, 0, None, 10, 10, 256, 256, 256, None, 256, 0, None) == N.ERR_INVALID_ARGUMENT
    assert f(1, None, 0, None, 10, 10, 256, 256, 256, None, 256, 0, None) == N.ERR_INVALID_ARGUMENT
    assert f(1, 256, 0, None, 10, 10, 256, 256, 256, None, None, 0, None) == N.ERR_INVALID_ARGUMENT
    assert f(1, 256, 0, 256, 10, 10, 256, 256, 256, None, 256, 0, None) == N.ERR_INVALID_ARGUMENT  # packs < 1
    assert f(1, 256, 0, None, 10, 10, 256, None, 256, None, 256, 0, None) == N.ERR_INVALID_ARGUMENT  # no adj
    assert f(1, 256, 0, None, 10, 10, 256, 256, 256, None, 256, N.FLAG_VALIDATE, None) == N.ERR_INVALID_ARGUMENT
    assert f(1, 256, 0, None, 10, 10, 256, 256, 256, None, 256, 1 << N.TUNE_RULER_SHIFT, None) \
        == N.ERR_INVALID_ARGUMENT  # tuning fields belong to the general path
    assert f(1, 256, 0, None, 1 << 30, 10, 256, 256, 256, None, 256, 0, None) == N.ERR_TOO_LARGE
    assert f(1, 256, 0, None, 10, (1 << 31) - 64, 256, 256, 256, None, 256, 0, None) == N.ERR_TOO_LARGE
    assert f(1, 256, 0, None, -1, 10, 256, 256, 256, None, 256, 0, None) == N.ERR_INVALID_ARGUMENT


@pytest.mark.parametrize("code", range(7))
def test_status_strings(code):
    s = N.lib().fastbcc_status_string(code).decode()
    assert s and s != "unknown status"


def test_tune_flag_encoding():
    assert N.tune_flags() == 0
    f = N.tune_flags(ruler_shift=6, sample_rounds=0, tile_shift=3)
    assert (f >> N.TUNE_RULER_SHIFT) & 0xF == 6
    assert (f >> N.TUNE_SAMPLE_SHIFT) & 0x3 == 3
    assert (f >> N.TUNE_TILE_SHIFT) & 0x7 == 3
    assert f & N.TUNE_CC_PRIORITY == 0
    assert N.tune_flags(cc_priority=True) == N.TUNE_CC_PRIORITY
    assert N.tune_flags(ldd=2) == 2 << N.TUNE_LDD_SHIFT
    assert N.tune_flags(sampled_tags=True) == N.TUNE_SAMPLED_TAGS
    assert (N.tune_flags(tag_samples=2) >> N.TUNE_TAG_SAMPLES_SHIFT) & 0x3 == 1
    assert (N.tune_flags(vertex_block=512) >> N.TUNE_VERTEX_BLOCK_SHIFT) & 0x3 == 3
    assert N.tune_flags(vertex_block=256) == 0
    assert N.tune_flags(compress_free_round=True) == N.TUNE_COMPRESS_FREE_ROUND
    assert N.tune_flags(xcd_order=True) == N.TUNE_XCD_ORDER
    assert N.tune_flags(graph_cc=True) == N.TUNE_GRAPH_CC == 1 << 31  # the last free bit: every bit has a meaning


def test_host_tensors_are_refused_not_solved_on_the_cpu():
    """The package has no CPU path: host tensors raise before any work."""
    import torch

    from paper_2301_01356_amd import solve, solve_batched

    off = torch.tensor([0, 1, 2], dtype=torch.int32)
    adj = torch.tensor([1, 0], dtype=torch.int32)
    with pytest.raises(ValueError, match="GPU"):
        solve(off, adj)
    with pytest.raises(ValueError, match="GPU"):
        solve_batched(torch.tensor([0, 2], dtype=torch.int32), off, adj)


def test_host_workspace_vbegin_and_outputs_are_refused():
    """A host workspace, a host vbegin or host outputs would hand host
    pointers to the kernels: every wrapper refuses them before any call."""
    import torch

    from paper_2301_01356_amd import api, read_device_status, solve_traced, vertex_labels

    host_ws = torch.empty(1 << 16, dtype=torch.uint8)
    with pytest.raises(ValueError, match="GPU"):
        api._check_workspace(host_ws, 2, 2, 1, None)
    with pytest.raises(ValueError, match="GPU"):
        vertex_labels(host_ws, 2, 2)
    with pytest.raises(ValueError, match="GPU"):
        read_device_status(host_ws)
    off = torch.tensor([0, 1, 2], dtype=torch.int32)
    adj = torch.tensor([1, 0], dtype=torch.int32)
    with pytest.raises(ValueError, match="GPU"):
        solve_traced(off, adj, None, vbegin=torch.tensor([0, 2], dtype=torch.int32))
    with pytest.raises(ValueError, match="GPU"):
        api._check_tensor(torch.tensor([0, 2], dtype=torch.int32), "vbegin", (torch.int32,))
    out = api.BccResult(torch.empty(2, dtype=torch.int32), torch.empty(2, dtype=torch.uint8),
                        torch.empty(1, dtype=torch.int64))
    with pytest.raises(ValueError, match="GPU"):
        api._check_result(out, 2, 2, 1, None)


def test_binding_constants_match_the_header():
    """Every FASTBCC_FLAG_* / FASTBCC_TUNE_* define and status code of the
    header has the same value in the Python binding."""
    text = open(HEADER).read()
    defines = dict(re.findall(r"#define\s+FASTBCC_((?:FLAG|TUNE)_\w+)\s+(0x[0-9a-fA-F]+|\d+)u?\b", text))
    assert defines, "no flag defines found"
    for name, value in defines.items():
        assert getattr(N, name) == int(value, 0), name
    statuses = dict(re.findall(r"\bFASTBCC_(OK|ERR_\w+)\s*=\s*(\d+)", text))
    assert statuses, "no status codes found"
    for name, value in statuses.items():
        assert getattr(N, name) == int(value), name
