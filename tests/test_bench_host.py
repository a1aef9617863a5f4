"""Host-side logic of bench.py, on the CPU: the one-GPU guard, the per-kernel
byte models behind the roofline figure, and the recorded counter table."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2301_01356_amd import _native as N  # noqa: E402


def _run_bench(args, **env):
    e = dict(os.environ, **env)
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=300, env=e, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run_bench(["--gpus", "2"])
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""  # no result line


def test_a_multi_rank_launch_is_refused():
    r = _run_bench([], WORLD_SIZE="2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_row_fill_model():
    n, A = 1000, 8000
    # offsets, one label store per arc, one (label, exact flag) pair per row
    assert bench.alg_bytes("k_bcc_rows", n, A) == 4 * (n + 1) + 4 * A + 8 * n
    assert bench.alg_bytes("k_no_such_kernel", n, A) is None


@pytest.mark.parametrize("ks", [1, 2, 3, 4])
def test_sampled_tag_model_counts_min_of_degree_and_samples(ks):
    deg = np.array([0, 1, 2, 3, 5, 100])
    flags = N.tune_flags(sampled_tags=True, tag_samples=ks)
    n = deg.size
    want = 28 * n + 8 * sum(min(int(d), ks) for d in deg)
    assert bench.alg_bytes("k_tag_sample", n, int(deg.sum()), deg, flags) == want


def test_sampling_round_model_counts_vertices_with_arcs():
    deg = np.array([0, 0, 3, 1])
    assert bench.alg_bytes("k_cc_sample", 4, 4, deg, 0) == 4 * 5 + 16 * 2


def test_recorded_counters_are_whole():
    c = bench.COUNTERS
    assert c["copy_factor"]["fetch"] > 0 and c["copy_factor"]["write"] > 0
    kernels = {k: v for k, v in c.items() if isinstance(v, dict) and "fetch_kib" in v}
    assert "k_tag_sample" in kernels and "k_bcc_rows" in kernels
    for k, v in kernels.items():
        assert v["fetch_kib"] > 0 and v["write_kib"] > 0, k
    # the row fill writes one 4-byte label per arc of R-MAT scale 25: its
    # write counter cannot be below that
    assert kernels["k_bcc_rows"]["write_kib"] * 1024 >= 4 * 1_047_198_154
    assert len(c["src_sha"]) == 16


def test_random_access_models():
    deg = np.array([0, 1, 2, 3, 5, 100])
    flags = N.tune_flags(sampled_tags=True, tag_samples=2)
    # first[] of min(deg, 2) neighbours per row plus one slot write per vertex with arcs
    assert bench.random_accesses("k_tag_sample", 6, int(deg.sum()), deg, flags) == (0 + 1 + 2 + 2 + 2 + 2) + 5
    assert bench.random_accesses("k_cc_sample", 6, int(deg.sum()), deg, flags) == 3 * 5
    assert bench.random_accesses("k_bcc_rows", 6, int(deg.sum()), deg, flags) is None
    assert bench.random_accesses("k_tag_sample", 6, 0) is None
