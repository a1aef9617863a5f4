"""The oracle's pins must catch plausible mistakes in it.

Each case compiles a copy of the C oracle with one planted mistake (on the
CPU, into a temporary directory) and checks that the brute-force pins from
``test_oracle`` reject it.
"""
import ctypes
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2301_01356_amd import gen
from tests import bruteforce as bf

MUTANTS = {
    "strict_fence_test": ("if (low[v] >= first[p]) {", "if (low[v] > first[p]) {"),
    "no_reverse_skip": ("if (fin[depth] >= 0 && a == rev[fin[depth]]) continue;", ""),
    "low_overwrite": ("if (first[w] < low[v]) low[v] = first[w];", "low[v] = first[w];"),
    "no_low_propagation": ("if (low[v] < low[p]) low[p] = low[v];", ""),
    "root_rule_off_by_one": ("else if (++root_children >= 2)", "else if (++root_children >= 1)"),
    "label_not_edge_id": ("int64_t id = e < rev[e] ? e : rev[e];", "int64_t id = e;"),
    "ap_for_root_always": ("if (depth > 0) out_ap[p] = 1;", "if (depth >= 0) out_ap[p] = 1;"),
}


def _build_mutant(tmp_path, name):
    src = open(oracle.SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, name
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / f"lib{name}.so"
    subprocess.run(["gcc", "-O1", "-std=c99", "-D_POSIX_C_SOURCE=199309L", "-shared", "-fPIC", str(path), "-o", str(lib)], check=True)
    return str(lib)


def _cases():
    rng = np.random.default_rng(77)
    out = []
    for _ in range(300):
        n = int(rng.integers(2, 9))
        m = int(rng.integers(1, 13))
        edges = [(int(rng.integers(0, n)), int(rng.integers(0, n))) for _ in range(m)]
        if rng.random() < 0.3:
            edges.append(edges[0])
        out.append(gen.multigraph_csr(n, edges))
    return out


def check_library(lib_path):
    """Exit status 1 if the library at ``lib_path`` disagrees with brute force
    on some case, 0 if it survives every case (run in a child process, so a
    mutant that crashes counts as caught too)."""
    h = ctypes.CDLL(lib_path)
    h.ht_bcc.restype = ctypes.c_int
    h.ht_bcc.argtypes = [ctypes.c_int64] + [ctypes.c_void_p] * 7
    for g in _cases():
        lab = np.empty(g.num_arcs, np.int32)
        ap = np.empty(g.n, np.uint8)
        nb = ctypes.c_int64(0)
        rc = h.ht_bcc(g.n, g.offsets.ctypes.data, g.adj.ctypes.data, lab.ctypes.data, ap.ctypes.data,
                      ctypes.addressof(nb), None, None)
        elab, eap, enb = bf.expected_from_csr(g.n, g.offsets, g.adj)
        if rc != 0 or nb.value != enb or not np.array_equal(lab, elab) or not np.array_equal(ap, eap):
            return 1
    return 0


def _child(lib_path):
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = f"import sys; sys.path.insert(0, {root!r}); from tests import test_oracle_mutants as t; sys.exit(t.check_library({lib_path!r}))"
    return subprocess.run([sys.executable, "-c", code], capture_output=True, timeout=300).returncode


def test_unmodified_oracle_survives():
    assert _child(oracle.LIB_PATH if os.path.exists(oracle.LIB_PATH) else oracle.build()) == 0


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_oracle_mistake_is_caught(tmp_path, name):
    assert _child(_build_mutant(tmp_path, name)) != 0, f"mutant {name} survived the brute-force pins"
