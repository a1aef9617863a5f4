"""CPU oracle for biconnected components -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports it, and the two share no code.

``ht_bcc`` runs the sequential Hopcroft-Tarjan algorithm (paper, Section
"Existing BCC Algorithms", "The Hopcroft-Tarjan Algorithm") written in plain C
(``ht_bcc.c``) on one host core, and returns the canonical edge partition:
every arc labelled by the smallest edge id (= smallest arc index) of its BCC,
-1 for self-loops, plus the articulation-point flags and the BCC count.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "ht_bcc.c")
LIB_PATH = os.path.join(_HERE, "libhtbcc.so")
_lib = None


def build() -> str:
    """Compile the C oracle into ``libhtbcc.so`` (plain gcc, one thread)."""
    cmd = ["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=199309L", "-shared", "-fPIC", SRC, "-o", LIB_PATH]
    subprocess.run(cmd, check=True)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        lib = ctypes.CDLL(LIB_PATH)
        lib.ht_bcc.restype = ctypes.c_int
        lib.ht_bcc.argtypes = [ctypes.c_int64] + [ctypes.c_void_p] * 7
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    pass


def ht_bcc(offsets, adj):
    """Hopcroft-Tarjan on a symmetric CSR.

    Returns ``(label int32[A], ap uint8[n], num_bcc, prep_seconds, ht_seconds)``.
    """
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    a = np.ascontiguousarray(adj, dtype=np.int32)
    n = off.shape[0] - 1
    if off[-1] != a.shape[0]:
        raise OracleError("offsets[n] != len(adj)")
    label = np.empty(a.shape[0], np.int32)
    ap = np.empty(n, np.uint8)
    nb = ctypes.c_int64(0)
    tp = ctypes.c_double(0)
    th = ctypes.c_double(0)
    rc = _load().ht_bcc(
        n,
        off.ctypes.data,
        a.ctypes.data,
        label.ctypes.data,
        ap.ctypes.data,
        ctypes.addressof(nb),
        ctypes.addressof(tp),
        ctypes.addressof(th),
    )
    if rc == -1:
        raise OracleError("CSR is not symmetric or has out-of-range ids")
    if rc != 0:
        raise OracleError(f"oracle failed ({rc})")
    return label, ap, int(nb.value), float(tp.value), float(th.value)
