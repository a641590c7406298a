"""Algorithmic HBM bytes of the solver's kernels.

Counting rule: the SpMV layout is read once per product; every row-indexed
float64 vector a kernel needs is read once and every vector it updates is
written once (8 bytes per row each); vectors gathered at neighbouring rows
are counted once (the extra gathers hit the caches).  Vectors that the
algorithms define as M^{-1} v are recomputed from the Jacobi diagonal d and
count as a read of d.
"""
from __future__ import annotations

# (reads, writes) in float64 words per row, per kernel, per variant and
# preconditioning (True = Jacobi).  "matrix" marks the kernel reading A.
KERNEL_WORDS = {
    ("hs", False): [("k_hs_xr", 4, 2, False), ("k_hs_p", 2, 1, False), ("k_hs_spmv", 1, 1, True)],
    ("hs", True): [("k_hs_xr", 5, 2, False), ("k_hs_p", 3, 1, False), ("k_hs_spmv", 1, 1, True)],
    ("pr", False): [("k_pr_update", 4, 3, False), ("k_pr_spmv", 2, 1, True)],
    ("pr", True): [("k_pr_update", 6, 4, False), ("k_pr_spmv", 4, 1, True)],
    ("pipe_pr", False): [("k_pipe_update", 6, 4, False), ("k_pipe_spmv", 2, 2, True)],
    ("pipe_pr", True): [("k_pipe_update", 9, 6, False), ("k_pipe_spmv", 2, 2, True)],
    # GV-CG: the direction updates of k-1 and the updates of k in one pass
    ("gv", False): [("k_gv_update", 7, 6, False), ("k_gv_spmv", 1, 1, True)],
    ("gv", True): [("k_gv_update", 10, 9, False), ("k_gv_spmv", 1, 1, True)],
    # CG-CG: direction updates of k-1 and updates of k in one pass; w = A r~
    ("cg", False): [("k_cg_update", 5, 4, False), ("k_cg_spmv", 1, 1, True), ("k_cg_finish", 0, 0, False)],
    ("cg", True): [("k_cg_update", 6, 5, False), ("k_cg_spmv", 1, 1, True), ("k_cg_finish", 0, 0, False)],
}
# fused structure (one kernel per PR / pipe-PR iteration, two per HS):
# neighbour recomputation reads each double-buffered vector once
KERNEL_WORDS_FUSED = {
    ("hs", False): [("k_hs_xr", 4, 2, False), ("k_hs_fused", 2, 2, True)],
    ("hs", True): [("k_hs_xr", 5, 2, False), ("k_hs_fused", 3, 2, True)],
    ("pr", False): [("k_pr_fused", 4, 4, True)],
    ("pr", True): [("k_pr_fused", 6, 5, True)],
    ("pipe_pr", False): [("k_pipe_fused", 6, 6, True)],
    ("pipe_pr", True): [("k_pipe_fused", 9, 8, True)],
}
# textbook HS-CG: one kernel per line of Alg. 1 (a dot of a vector with
# itself reads it once)
KERNEL_WORDS_TEXTBOOK = {
    ("hs", False): [("k_tb_mu", 0, 0, False), ("k_tb_axpy_x", 2, 1, False), ("k_tb_axpy_r", 2, 1, False),
                    ("k_tb_dot_nu", 1, 0, False), ("k_tb_nu", 0, 0, False), ("k_tb_xpay_p", 2, 1, False),
                    ("k_tb_spmv", 1, 1, True), ("k_tb_dot_mu", 2, 0, False)],
    ("hs", True): [("k_tb_mu", 0, 0, False), ("k_tb_axpy_x", 2, 1, False), ("k_tb_axpy_r", 2, 1, False),
                   ("k_tb_prec", 2, 1, False), ("k_tb_dot_nu", 2, 0, False), ("k_tb_dot_rr", 1, 0, False),
                   ("k_tb_nu", 0, 0, False), ("k_tb_xpay_p", 2, 1, False), ("k_tb_spmv", 1, 1, True),
                   ("k_tb_dot_mu", 2, 0, False)],
}
for _tab in (KERNEL_WORDS_FUSED,):
    for _j in (False, True):
        _tab[("m", _j)] = _tab[("pr", _j)]
        _tab[("pipe_m", _j)] = _tab[("pipe_pr", _j)]
# pipe-PR-CG without the recompute of w: the update also writes w' (and
# reads/writes w~' with Jacobi); the product reads only s~ of the pair
KERNEL_WORDS[("pipe_pr_nowrecompute", False)] = [("k_pipe_update", 6, 5, False), ("k_pipe_spmv", 2, 1, True)]
KERNEL_WORDS[("pipe_pr_nowrecompute", True)] = [("k_pipe_update", 10, 8, False), ("k_pipe_spmv", 2, 1, True)]
# PR-CG with eq. nuk: with Jacobi the product also reads r for delta = <s~, r>
KERNEL_WORDS[("pr_unsimplified", False)] = KERNEL_WORDS[("pr", False)]
KERNEL_WORDS[("pr_unsimplified", True)] = KERNEL_WORDS[("pr", True)]
KERNEL_WORDS[("pr_norecompute", False)] = KERNEL_WORDS[("pr", False)]
KERNEL_WORDS[("pr_norecompute", True)] = KERNEL_WORDS[("pr", True)]
KERNEL_WORDS[("m", False)] = KERNEL_WORDS[("pr", False)]
KERNEL_WORDS[("m", True)] = KERNEL_WORDS[("pr", True)]
KERNEL_WORDS[("pipe_m", False)] = KERNEL_WORDS[("pipe_pr", False)]
KERNEL_WORDS[("pipe_m", True)] = KERNEL_WORDS[("pipe_pr", True)]


def kernel_bytes(variant: str, jacobi: bool, n: int, matrix_bytes: int, fused: bool = False,
                 textbook: bool = False, nu_in_update: bool = False) -> dict:
    """Algorithmic bytes per launch of each kernel of one iteration.

    nu_in_update: PR/M with Jacobi, where the update kernel forms <r~, r> and
    <r, r> from the rows it writes, so the product kernel does not read r."""
    out = {}
    table = KERNEL_WORDS_TEXTBOOK if textbook else (KERNEL_WORDS_FUSED if fused else KERNEL_WORDS)
    for name, r, w, mat in table[(variant, jacobi)]:
        if nu_in_update and jacobi and not fused and name == "k_pr_spmv" and variant != "pr_unsimplified":
            r -= 1
        out[name] = 8 * n * (r + w) + (matrix_bytes if mat else 0)
    return out


def iteration_bytes(variant: str, jacobi: bool, n: int, matrix_bytes: int, fused: bool = False,
                    textbook: bool = False, nu_in_update: bool = False) -> int:
    return sum(kernel_bytes(variant, jacobi, n, matrix_bytes, fused, textbook, nu_in_update).values())


def csr_matrix_bytes(n: int, nnz: int) -> int:
    """Bytes of plain CSR (int32 indices, float64 values) read once."""
    return 12 * nnz + 4 * (n + 1)


def batched_words(mode: str, fused: bool, jacobi: bool = False) -> int:
    """Vector words per row and iteration of a batched PR-CG solve: the fused
    lockstep iteration reads x, r, p, s and writes x, r', p', s' (with Jacobi
    also r~ and d read and r~' written); the three-launch lockstep iteration
    and the persistent kernel move the two-kernel byte model's words (the
    update reads x, r, p, s and writes x, r, p; the product reads p, r and
    writes s; with Jacobi r~ and d as well)."""
    if mode == "lockstep" and fused:
        return 12 if jacobi else 8
    return 15 if jacobi else 10


def batched_bytes(row_iterations: float, words: int, matrix_bytes: int, n: int, nnz: int) -> tuple:
    """Bytes moved by a batched solve of sum over systems of (iterations x
    rows) = row_iterations: per row and iteration the vector words plus the
    system's share of the matrix, taken per row, either as the batch's own
    storage (matrix_bytes, read once per iteration of every system) or as
    the CSR count 12 nnz + 4 (n + 1).  Returns (format bytes, CSR bytes)."""
    fmt = row_iterations * (8.0 * words + matrix_bytes / float(n))
    csr = row_iterations * (8.0 * words + csr_matrix_bytes(n, nnz) / float(n))
    return fmt, csr
