"""Host-side checks of the benchmark and its byte model (no GPU)."""
import json
import os
import subprocess
import sys

import pytest

from paper_1905_01549_amd import traffic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
N128 = 128 ** 3


def test_bench_refuses_several_gpus():
    """One GPU only: --gpus above 1 exits with a message before touching a GPU."""
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in json.loads(p.stdout.strip().splitlines()[-1])["error"]


@pytest.mark.parametrize("variant, jacobi, words", [
    # Alg. 2 with Jacobi: update reads s, p, x, r, r~, d and writes x, r, r~, p;
    # the product reads p, r, r~, d (mu, sigma, gamma, nu, <r, r>) and writes s
    ("pr", True, 6 + 4 + 4 + 1),
    # without a preconditioner r~ = r and s~ = s are not stored
    ("pr", False, 4 + 3 + 2 + 1),
    # Alg. 1: x, r (reads s, p, x, r, d) then p (reads r, d, p), then s = A p
    ("hs", True, 5 + 2 + 3 + 1 + 1 + 1),
    # Alg. 3 with Jacobi: update of x, r, r~, p, s, s~, w', w~' and the dots;
    # one pass over A for (u, w) = A (s~, r~)
    ("pipe_pr", True, 9 + 6 + 2 + 2),
])
def test_byte_model_counts_each_algorithms_vectors(variant, jacobi, words):
    assert traffic.iteration_bytes(variant, jacobi, N128, 0) == 8 * N128 * words
    assert traffic.iteration_bytes(variant, jacobi, N128, 1000) == 8 * N128 * words + 1000  # A read once


@pytest.mark.parametrize("variant, kw, words", [
    ("pr", {"nu_in_update": True}, 14),   # the benchmark's PR-CG: the update forms nu and <r, r>
    ("hs", {}, 13),
    ("pipe_pr", {}, 19),
    ("cg", {}, 13),
    ("hs", {"textbook": True}, 19),       # one kernel per line of Alg. 1
    ("pr", {"fused": True}, 11),          # one kernel per iteration
])
def test_byte_model_words_per_iteration_with_jacobi(variant, kw, words):
    """Vector words per row per iteration besides one read of A (the
    353.1 / 336.3 / 437.0 / 336.3 / 437.0 / 302.8 MB per iteration of the
    128^3 benchmark with its 118.2 MB matrix)."""
    mb = 118_200_000
    assert traffic.iteration_bytes(variant, True, N128, mb, **kw) - mb == 8 * N128 * words


def test_traffic_of_an_unprofiled_workload_is_none():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.load_traffic("k_pr_spmv", "no_such_workload") is None


@pytest.mark.parametrize("mode, fused, jacobi, words", [
    ("lockstep", True, False, 8),     # x, r, p, s read; x, r', p', s' written
    ("lockstep", True, True, 12),     # and r~, d read, r~' written
    ("lockstep", False, False, 10),   # update 4 + 3, product 2 + 1
    ("persistent", False, False, 10),
    ("persistent", True, True, 15),   # fusion applies to the lockstep mode only
])
def test_batched_words_follow_the_structure(mode, fused, jacobi, words):
    assert traffic.batched_words(mode, fused, jacobi) == words


def test_batched_bytes_take_the_matrix_per_row():
    """Two systems of 100 and 300 rows running 10 and 20 iterations: 7,000
    row-iterations, each with its words and the matrix's bytes per row, in
    the batch's own storage or as the CSR count."""
    n, nnz, matrix_bytes = 400, 2000, 16_000
    fmt, csr = traffic.batched_bytes(100 * 10 + 300 * 20, 8, matrix_bytes, n, nnz)
    assert fmt == 7000 * (64 + 40)
    assert csr == 7000 * (64 + (12 * 2000 + 4 * 401) / 400)
