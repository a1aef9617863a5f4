"""ctypes binding of ``libfastbcc.so`` (the C ABI in ``include/fastbcc.h``).

Argument marshalling only: every step of the solve runs in the HIP kernels of
the library.  If the library is missing the import fails loudly; there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfastbcc.so")

# status codes (fastbcc_status)
OK = 0
ERR_INVALID_ARGUMENT = 1
ERR_TOO_LARGE = 2
ERR_WORKSPACE_TOO_SMALL = 3
ERR_HIP = 4
ERR_INVALID_GRAPH = 5
ERR_SCRATCH_TOO_SMALL = 6
NOALLOC_SCRATCH_BYTES = 64 << 20  # FASTBCC_NOALLOC_SCRATCH_BYTES
SMALL_MAX_VERTICES = 3072  # FASTBCC_SMALL_MAX_VERTICES

FLAG_VALIDATE = 0x1
FLAG_SORTED_ROWS = 0x2
FLAG_NO_SELF_LOOPS = 0x4
FLAG_REPAIR = 0x8
TUNE_RULER_SHIFT = 8
TUNE_SAMPLE_SHIFT = 12
TUNE_TILE_SHIFT = 14
TUNE_CC_PRIORITY = 0x20000
TUNE_LDD_SHIFT = 18
TUNE_SAMPLED_TAGS = 0x100000
TUNE_TAG_SAMPLES_SHIFT = 21
TAG_SAMPLE_CODES = {4: 0, 2: 1, 3: 2, 1: 3}
TUNE_FREE_FIRST_ROUND = 0x800000
TUNE_LCC_PRIORITY = 0x1000000
TUNE_LCC_ROUNDS_SHIFT = 25
TUNE_VERTEX_BLOCK_SHIFT = 27
TUNE_COMPRESS_FREE_ROUND = 0x20000000
TUNE_XCD_ORDER = 0x40000000
TUNE_GRAPH_CC = 0x80000000
VERTEX_BLOCK_CODES = {256: 0, 64: 1, 128: 2, 512: 3}

EXPORTED = (
    "fastbcc_workspace_size",
    "fastbcc_solve",
    "fastbcc_solve_off64",
    "fastbcc_solve_batched",
    "fastbcc_read_device_status",
    "fastbcc_status_string",
    "fastbcc_version",
    "fastbcc_solve_traced",
    "fastbcc_trace_create",
    "fastbcc_trace_destroy",
    "fastbcc_trace_collect",
    "fastbcc_trace_count",
    "fastbcc_trace_entry",
    "fastbcc_trace_dropped",
    "fastbcc_trace_reset",
    "fastbcc_vertex_labels",
    "fastbcc_solve_noalloc",
    "fastbcc_bc_labeling",
    "fastbcc_check_batched",
    "fastbcc_batch_rebase",
    "fastbcc_solve_small",
)


class FastBccError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = lib().fastbcc_status_string(status).decode() if _lib is not None else str(status)
        super().__init__(f"{what}: {msg} (status {status})" if what else f"{msg} (status {status})")


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2301_01356_amd.build` "
            "(there is no non-HIP fallback)"
        )
    h = ctypes.CDLL(LIB_PATH)
    i64, i32, u32, vp, sz = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_size_t
    st = ctypes.c_int
    h.fastbcc_workspace_size.restype = st
    h.fastbcc_workspace_size.argtypes = [i64, i64, i32, ctypes.POINTER(sz)]
    solve_args = [i64, i64, vp, vp, vp, vp, vp, vp, sz, u32, vp]
    h.fastbcc_solve.restype = st
    h.fastbcc_solve.argtypes = solve_args
    h.fastbcc_solve_off64.restype = st
    h.fastbcc_solve_off64.argtypes = solve_args
    h.fastbcc_solve_batched.restype = st
    h.fastbcc_solve_batched.argtypes = [i32, vp, i64, i64, vp, vp, vp, vp, vp, vp, sz, u32, vp]
    h.fastbcc_read_device_status.restype = st
    h.fastbcc_read_device_status.argtypes = [vp, vp, ctypes.POINTER(i32)]
    h.fastbcc_status_string.restype = ctypes.c_char_p
    h.fastbcc_status_string.argtypes = [st]
    h.fastbcc_version.restype = ctypes.c_char_p
    h.fastbcc_version.argtypes = []
    h.fastbcc_solve_traced.restype = st
    h.fastbcc_solve_traced.argtypes = [i32, vp, i64, i64, vp, i32, vp, vp, vp, vp, vp, sz, u32, vp, vp]
    h.fastbcc_trace_create.restype = vp
    h.fastbcc_trace_create.argtypes = [i32]
    h.fastbcc_trace_destroy.restype = None
    h.fastbcc_trace_destroy.argtypes = [vp]
    h.fastbcc_trace_collect.restype = st
    h.fastbcc_trace_collect.argtypes = [vp]
    h.fastbcc_trace_count.restype = i32
    h.fastbcc_trace_count.argtypes = [vp]
    h.fastbcc_trace_entry.restype = st
    h.fastbcc_trace_entry.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(i64)]
    h.fastbcc_trace_dropped.restype = i64
    h.fastbcc_trace_dropped.argtypes = [vp]
    h.fastbcc_trace_reset.restype = None
    h.fastbcc_trace_reset.argtypes = [vp]
    h.fastbcc_solve_noalloc.restype = st
    h.fastbcc_solve_noalloc.argtypes = [i64, i64, vp, vp, vp, vp, vp, u32, vp]
    h.fastbcc_bc_labeling.restype = st
    h.fastbcc_bc_labeling.argtypes = [i64, i64, i32, vp, vp, i32, vp, vp, vp, vp, sz, u32, vp, vp, vp, vp, vp]
    h.fastbcc_batch_rebase.restype = st
    h.fastbcc_batch_rebase.argtypes = [i32, vp, vp, i64, i64, vp, vp, vp]
    h.fastbcc_check_batched.restype = st
    h.fastbcc_check_batched.argtypes = [i32, vp, i64, i64, vp, vp, u32, vp, vp]
    h.fastbcc_solve_small.restype = st
    h.fastbcc_solve_small.argtypes = [i32, vp, i32, vp, i64, i64, vp, vp, vp, vp, vp, u32, vp]
    h.fastbcc_vertex_labels.restype = st
    h.fastbcc_vertex_labels.argtypes = [i64, i64, i32, vp, vp, sz, vp, vp, vp]
    _lib = h
    return h


def check(status: int, what: str = "") -> None:
    if status != OK:
        raise FastBccError(status, what)


def workspace_size(n: int, num_arcs: int, num_graphs: int = 1) -> int:
    out = ctypes.c_size_t(0)
    check(lib().fastbcc_workspace_size(int(n), int(num_arcs), int(num_graphs), ctypes.byref(out)), "workspace_size")
    return int(out.value)


def tune_flags(ruler_shift: int = 0, sample_rounds=None, tile_shift: int = 0, cc_priority: bool = False,
               ldd: int = 0, sampled_tags: bool = False, tag_samples: int = 4,
               free_first_round: bool = False, lcc_priority: bool = False, lcc_rounds=None,
               vertex_block: int = 256, compress_free_round: bool = False, xcd_order: bool = False,
               graph_cc: bool = False) -> int:
    """Encode tuning fields (0/None = library default).  ``ldd`` = k turns on
    the low-diameter decomposition before First-CC's union-find, beta = 2^-k;
    ``sampled_tags`` certifies fences from ``tag_samples`` (1, 2, 3 or 4)
    sampled neighbours per vertex first; ``vertex_block`` (64, 128, 256 or
    512) is the block size of the hot per-vertex kernels; ``graph_cc`` runs a
    batch's First-CC per graph, one workgroup each."""
    f = TUNE_CC_PRIORITY if cc_priority else 0
    f |= TUNE_SAMPLED_TAGS if sampled_tags else 0
    f |= TAG_SAMPLE_CODES[tag_samples] << TUNE_TAG_SAMPLES_SHIFT
    f |= TUNE_FREE_FIRST_ROUND if free_first_round else 0
    f |= TUNE_LCC_PRIORITY if lcc_priority else 0
    if lcc_rounds is not None:
        f |= (int(lcc_rounds) + 1) << TUNE_LCC_ROUNDS_SHIFT
    f |= (ldd & 0x3) << TUNE_LDD_SHIFT
    f |= VERTEX_BLOCK_CODES[vertex_block] << TUNE_VERTEX_BLOCK_SHIFT
    f |= TUNE_COMPRESS_FREE_ROUND if compress_free_round else 0
    f |= TUNE_XCD_ORDER if xcd_order else 0
    f |= TUNE_GRAPH_CC if graph_cc else 0
    if ruler_shift:
        f |= (ruler_shift & 0xF) << TUNE_RULER_SHIFT
    if sample_rounds is not None:
        f |= (3 if sample_rounds == 0 else sample_rounds) << TUNE_SAMPLE_SHIFT
    if tile_shift:
        f |= (tile_shift & 0x7) << TUNE_TILE_SHIFT
    return f


class Trace:
    """Per-kernel HIP-event timing over any number of traced solves."""

    def __init__(self, max_launches: int = 8192):
        self.h = lib().fastbcc_trace_create(int(max_launches))
        if not self.h:
            raise FastBccError(ERR_HIP, "fastbcc_trace_create")

    def collect(self) -> None:
        check(lib().fastbcc_trace_collect(self.h), "fastbcc_trace_collect")

    def totals(self) -> dict:
        """{kernel name: (total ms, timed launches)} of everything collected.
        Template arguments are dropped from the names, so the variants of one
        kernel (e.g. the two union-find hooking rules) share an entry."""
        out = {}
        for i in range(lib().fastbcc_trace_count(self.h)):
            name = ctypes.c_char_p()
            ms = ctypes.c_double()
            nl = ctypes.c_int64()
            check(lib().fastbcc_trace_entry(self.h, i, ctypes.byref(name), ctypes.byref(ms), ctypes.byref(nl)))
            key = name.value.decode().split("<", 1)[0]
            t, c = out.get(key, (0.0, 0))
            out[key] = (t + ms.value, c + nl.value)
        return out

    def dropped(self) -> int:
        return int(lib().fastbcc_trace_dropped(self.h))

    def reset(self) -> None:
        lib().fastbcc_trace_reset(self.h)

    def close(self) -> None:
        if self.h:
            lib().fastbcc_trace_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
