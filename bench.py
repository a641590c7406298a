"""Benchmark: FP64 PR-CG iterations per second on the 3D 7-point Poisson
problem, 128^3 grid (n = 2,097,152, 14,581,760 nonzeros), Jacobi
preconditioner, b ~ U[-1,1].  One step = one solve from x0 = 0 to
||r_k|| <= 1e-10 ||b|| (at most 1000 iterations): the initialisation, the
iterations and the exit kernels.  Inputs are resident in HBM before timing
starts.

Prints one JSON line (see the repository's benchmark contract); extra keys:
per-variant timings (HS-CG, PR-CG, pipe-PR-CG), the dominant kernel's
roofline from HIP events around its launches, and the CPU oracle baseline
on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# kernel structures compared ("auto", the library's default, is "fused" for
# HS-CG and PR-CG below 2048 workgroups and otherwise "two_pass", which places
# stage 2 by size)
STRUCTURES = ("auto", "two_pass", "two_pass_redundant", "two_pass_stage2", "two_pass_last", "fused", "textbook")
TOL = 1e-10
MAXIT = 1000


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--variant", default="pr")
    ap.add_argument("--grid", type=int, default=0, help="override the workgroup count (tuning)")
    ap.add_argument("--kernels", default="auto", help="kernel structure of the flagship run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--m", type=int, default=128, help="grid edge (128 = the benchmark workload)")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only time the flagship variant's kernels (the launches the roofline uses)")
    ap.add_argument("--workload", default="poisson3d_128_jacobi", choices=("poisson3d_128_jacobi", "varcoef27_160"),
                    help="workload of --kernels-only (varcoef27_160: the 27-point 160^3 problem, no preconditioner)")
    ap.add_argument("--no-27pt", action="store_true", help="skip the 27-point 160^3 section")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--batched-only", action="store_true",
                    help="only the batched workload (both modes; one JSON line)")
    ap.add_argument("--batched-reps", type=int, default=3, help="timed batched solves per mode")
    ap.add_argument("--batched-config", default="",
                    help="threads,per_cu,slices_in_flight,group_slices fixed instead of autotuned "
                         "(0 leaves a part to the autotuner), so that profiled runs launch the same kernels")
    ap.add_argument("--batched-fusion", default="auto", choices=("auto", "off", "on"),
                    help="fused lockstep iterations: timed by the autotuner, never, or always")
    ap.add_argument("--no-sequential", action="store_true",
                    help="skip the 512 one-at-a-time solves of the batched comparison (profiling runs)")
    ap.add_argument("--suite", action="store_true",
                    help="per-iteration times of every variant on every workload (one JSON line each)")
    return ap.parse_args()


# the sources that define the single-system iteration kernels and their
# launch (the batched, fused, textbook and setup kernels are elsewhere)
DIGEST_SOURCES = ("kernels_iter.hip", "prcg_device.h", "prcg_common.h", "prcg_api.hip")


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1905_01549_amd", "csrc")
    for name in DIGEST_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str):
    """HBM bytes per launch measured with rocprofv3 counters, if they were
    taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_digest") != kernel_source_digest():
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def variants_of(kern: str):
    """Variants timed under a kernel structure (GV-CG, CG-CG and PR-CG with eq. nuk have one)."""
    if kern == "textbook":
        return ("hs",)
    if kern in ("auto", "two_pass"):
        return ("hs", "pr", "pipe_pr", "gv", "cg", "pr_unsimplified")
    return ("hs", "pr", "pipe_pr")


def nu_split(M) -> bool:
    """Whether PR's update kernel forms <r~, r> and <r, r> (Jacobi): stage 2
    outside the update kernel, i.e. in its own kernel or a last workgroup."""
    p = M.props
    return bool(p.stage2 & 2) or p.kernels == 4


def stream_triad(torch, n=64 * 1024 * 1024, reps=20):
    """A STREAM triad a = b + s c on three float64 arrays of 512 MiB each
    (beyond the 256 MB Infinity Cache), with torch's elementwise kernel: a
    measured reference bandwidth for the mix of two reads and one write, to
    set the kernels' GB/s against besides the 8 TB/s peak."""
    b = torch.rand(n, dtype=torch.float64, device="cuda")
    c = torch.rand(n, dtype=torch.float64, device="cuda")
    a = torch.empty_like(b)
    for _ in range(3):
        torch.add(b, c, alpha=3.0, out=a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        torch.add(b, c, alpha=3.0, out=a)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    del a, b, c
    return 3 * 8 * n / sec / 1e9


def calibration_copy(torch):
    """A plain device-to-device copy of known size (256 MiB read + 256 MiB
    written) to calibrate hardware byte counters against."""
    src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()


def device_facts(torch):
    """The properties the design assumes, as the runtime reports them."""
    pr = torch.cuda.get_device_properties(0)
    facts = {"name": pr.name, "arch": getattr(pr, "gcnArchName", None),
             "compute_units": pr.multi_processor_count, "memory_GiB": round(pr.total_memory / 2 ** 30, 1)}
    l2 = getattr(pr, "L2_cache_size", None)
    if l2:
        facts["l2_MiB"] = round(l2 / 2 ** 20, 2)
    return facts


def batched_section(torch, prcg, problems, traffic, reps=3, sequential=True, config="", fusion="auto"):
    """512 anisotropic systems in one batched solve (the mode the solver picks;
    both modes are timed) vs one prcg_solve per system."""
    A, offs, b, xs, eps = problems.config4()
    M = prcg.Matrix(A.row_ptr, A.col_idx, A.values, "none")
    B = prcg.Batch(M, offs)
    if config:
        B.set_config(*[int(v) for v in config.split(",")])
    B.set_fusion(fusion)
    bt = torch.as_tensor(b, device="cuda")
    x, iters, status = B.solve(bt, "pr", 1e-10, 20000)  # includes the autotuner's trial runs
    assert all(st == "ok" for st in status)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        x, iters, status = B.solve(bt, "pr", 1e-10, 20000)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t) / reps
    nt, grid = B.config("pr")
    mode = B.mode("pr")
    props = B.props("pr")  # the configuration the autotuner chose
    per_mode = {}
    for m in ("persistent", "lockstep"):
        B.set_mode(m)
        B.solve(bt, "pr", 1e-10, 20000)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            _, it_m, st_m = B.solve(bt, "pr", 1e-10, 20000)
        torch.cuda.synchronize()
        assert all(st == "ok" for st in st_m)
        per_mode[m] = {"solves_per_s": (len(offs) - 1) / ((time.perf_counter() - t) / reps),
                       "iterations_total": int(it_m.sum())}
    sizes = np.diff(offs)
    # algorithmic bytes per system-iteration: the vector words per row of the
    # structure that ran (8 for the fused lockstep iteration: x, r, p, s read
    # and written, p recomputed at the neighbouring rows; 10 otherwise: the
    # update reads x, r, p, s and writes x, r, p, the product reads p, r and
    # writes s) plus the system's share of the matrix, taken per row: the
    # batch's SELL-64 bytes (format basis) or the CSR count 12 nnz + 4 (n + 1)
    # of the byte model
    words = traffic.batched_words(mode, bool(props["fused"]))
    moved, moved_csr = traffic.batched_bytes(float(np.sum(iters * sizes)), words, props["matrix_bytes"], A.n, A.nnz)
    # sequential: one handle and one solve per system (handles created before timing)
    t_seq, seq_iters = float("nan"), 0
    if sequential:
        mats = [problems.batch_system(s_)[0] for s_ in range(len(sizes))]
        handles = [prcg.Matrix(m.row_ptr, m.col_idx, m.values, "none") for m in mats]
        bs = [bt[offs[s_]:offs[s_ + 1]].contiguous() for s_ in range(len(sizes))]
        torch.cuda.synchronize()
        t = time.perf_counter()
        for h, bb in zip(handles, bs):
            _, info = h.solve(bb, "pr", 1e-10, 20000)
            seq_iters += info.iters
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t
        for h in handles:
            h.close()
    B.close()
    M.close()
    return {"workload": "aniso2d_batch_512", "systems": int(len(sizes)), "n_total": int(A.n),
            "nnz_total": int(A.nnz), "batched_solves_per_s": len(sizes) / t_batch, "batched_ms": t_batch * 1e3,
            "sequential_solves_per_s": len(sizes) / t_seq if sequential else None,
            "sequential_ms": t_seq * 1e3 if sequential else None,
            "speedup": t_seq / t_batch if sequential else None, "iterations_total": int(iters.sum()), "sequential_iterations": seq_iters,
            "words_per_row": words, "algorithmic_GBps": moved / t_batch / 1e9,
            "hbm_frac": moved / t_batch / 1e9 / HBM_PEAK_GBS, "bytes_moved": moved,
            "algorithmic_GBps_csr_model": moved_csr / t_batch / 1e9,
            "hbm_frac_csr_model": moved_csr / t_batch / 1e9 / HBM_PEAK_GBS, "bytes_moved_csr_model": moved_csr,
            "mode": mode, "modes": per_mode, "threads_per_workgroup": nt, "workgroups": grid, "tuned": props}


def roofline_of(kernel_us, fmt_bytes, csr_bytes):
    """A kernel's achieved GB/s and fraction of peak on two byte counts: the
    bytes its own storage format must move (the SELL-64 layout: offset-aligned
    slices store no column index) and the CSR count of the byte model
    (12 nnz + 4 (n + 1) for the matrix), which overstates what this format
    reads."""
    sec = kernel_us * 1e-6
    return {"bytes_per_launch": fmt_bytes, "achieved": fmt_bytes / sec / 1e9,
            "frac": fmt_bytes / sec / 1e9 / HBM_PEAK_GBS,
            "bytes_per_launch_csr_model": csr_bytes, "achieved_csr_model": csr_bytes / sec / 1e9,
            "frac_csr_model": csr_bytes / sec / 1e9 / HBM_PEAK_GBS}


def varcoef27_section(torch, prcg, problems, traffic):
    """The 27-point variable-coefficient problem on 160^3 cells (n 4,096,000,
    nnz 109,215,352, lognormal(0,1) cell coefficients, no preconditioner),
    whose 1.2 GB iteration streams from HBM: complete solves to 1e-10 of
    HS-CG, PR-CG and pipe-PR-CG (best of 2, us per iteration and algorithmic
    GB/s over the iteration) and every kernel's full-work launch time (100
    iterations at tol = 0, HIP dispatch events)."""
    pr = problems.config3b()
    A = pr.A
    M = prcg.Matrix(A.row_ptr, A.col_idx, A.values, "none")
    b = torch.as_tensor(pr.b, device="cuda")
    props = M.props
    n = A.n
    csr = traffic.csr_matrix_bytes(n, A.nnz)
    out = {"workload": "varcoef27_160", "n": int(n), "nnz": int(A.nnz), "precond": "none", "tol": TOL,
           "matrix_bytes_format": int(props.matrix_bytes), "matrix_bytes_csr_model": int(csr),
           "grid": int(props.grid), "variants": {}}
    for v in ("hs", "pr", "pipe_pr"):
        _, info = M.solve(b, v, TOL, 20000)
        best = float("inf")
        for _ in range(2):
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, info = M.solve(b, v, TOL, 20000)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t)
        it_fmt = traffic.iteration_bytes(v, False, n, props.matrix_bytes)
        it_csr = traffic.iteration_bytes(v, False, n, csr)
        sec = best / max(info.iters, 1)
        kt = M.time_kernels(v, 100)
        kb = traffic.kernel_bytes(v, False, n, props.matrix_bytes)
        kc = traffic.kernel_bytes(v, False, n, csr)
        out["variants"][v] = {
            "iters": info.iters, "status": info.status, "relres_true": info.relres_true,
            "us_per_iter": sec * 1e6, "iters_per_s": 1.0 / sec,
            "bytes_per_iter": it_fmt, "algorithmic_GBps": it_fmt / sec / 1e9,
            "frac": it_fmt / sec / 1e9 / HBM_PEAK_GBS,
            "bytes_per_iter_csr_model": it_csr, "frac_csr_model": it_csr / sec / 1e9 / HBM_PEAK_GBS,
            "kernels": {k: {"us": ms * 1e3, **(roofline_of(ms * 1e3, kb[k], kc[k]) if k in kb else {})}
                        for k, ms in kt}}
    prk = out["variants"]["pr"]["kernels"]
    dom = max((k for k in prk if "bytes_per_launch" in prk[k]), key=lambda k: prk[k]["us"])
    out["dominant_kernel"] = {"kernel": dom, "us_per_launch": prk[dom]["us"], **{k: v for k, v in prk[dom].items()
                                                                                 if k != "us"},
                              "traffic": load_traffic(dom, "varcoef27_160")}
    M.close()
    return out


def unrolled_pr_cg(torch, rows, cols, vals, b, iters):
    """PR-CG (Alg. 2, no preconditioner) written with differentiable torch ops
    for a fixed number of iterations: the autograd-unrolling comparator."""
    n = b.shape[0]

    def spmv(v):
        return torch.zeros(n, dtype=v.dtype, device=v.device).index_add(0, rows, vals * v[cols])

    x = torch.zeros_like(b)
    r = b - spmv(x)
    p = r
    s = spmv(p)
    nu, mu, sigma, gamma = r @ r, p @ s, r @ s, s @ s
    for _ in range(iters):
        alpha = nu / mu
        x = x + alpha * p
        r = r - alpha * s
        nup = nu - 2.0 * alpha * sigma + alpha * alpha * gamma
        beta = nup / nu
        p = r + beta * p
        s = spmv(p)
        mu, sigma, gamma, nu = p @ s, r @ s, s @ s, r @ r
    return x


def adjoint_section(torch, prcg, problems):
    """Gradient of w^T x, x = A^{-1} b, w.r.t. b and the CSR values on the
    96^3 variable-coefficient problem: adjoint solve vs unrolled autograd."""
    from paper_1905_01549_amd.autograd import solve as dsolve
    pr = problems.config5()
    A = pr.A
    M = prcg.Matrix(A.row_ptr, A.col_idx, A.values, "none")
    w = torch.as_tensor(pr.extra["w"], device="cuda")
    vals0 = torch.as_tensor(A.values, device="cuda")
    b0 = torch.as_tensor(pr.b, device="cuda")

    def adjoint_grad(tol=1e-10):
        vals = vals0.clone().requires_grad_(True)
        b = b0.clone().requires_grad_(True)
        x = dsolve(vals, b, M, "pr", tol, 20000)
        (w * x).sum().backward()
        return vals.grad, b.grad

    def rel(g, ref):
        return float((g - ref).abs().max() / ref.abs().max())

    # reference gradients: forward and adjoint solves to 1e-13 (1e-12 if the
    # updated residual does not get there)
    try:
        ref_tol = 1e-13
        gv_ref, gb_ref = adjoint_grad(ref_tol)
    except RuntimeError:
        ref_tol = 1e-12
        gv_ref, gb_ref = adjoint_grad(ref_tol)
    gv, gb = adjoint_grad()
    err_adj = {"values": rel(gv, gv_ref), "b": rel(gb, gb_ref)}
    reps = 3
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        gv, gb = adjoint_grad()
    torch.cuda.synchronize()
    t_adj = (time.perf_counter() - t) / reps
    _, info = M.solve(b0, "pr", 1e-10, 20000)
    iters = info.iters
    rows = torch.as_tensor(np.repeat(np.arange(A.n), np.diff(A.row_ptr)), device="cuda")
    cols = torch.as_tensor(A.col_idx.astype(np.int64), device="cuda")

    def unrolled_grad(k):
        vals = vals0.clone().requires_grad_(True)
        b = b0.clone().requires_grad_(True)
        x = unrolled_pr_cg(torch, rows, cols, vals, b, k)
        (w * x).sum().backward()
        return vals.grad, b.grad

    # Equal accuracy: the unrolled gradients at the forward iteration count
    # and at twice that count, until both are as close to the reference
    # gradients (max relative difference) as the adjoint's are; the unrolled
    # graph keeps every iteration's vectors (about 120 MB per iteration
    # here), so a count whose predicted memory exceeds 0.6 of the free device
    # memory is not run.
    unrolled = {}
    unrolled_grad(iters)  # warm-up (allocator, kernels)
    matched = None
    for k in (iters, 2 * iters):
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        torch.cuda.reset_peak_memory_stats()
        base = torch.cuda.memory_allocated()
        free, _ = torch.cuda.mem_get_info()
        if unrolled:
            last = unrolled[max(unrolled)]
            if last["peak_bytes"] / last["iterations"] * k > 0.6 * free:
                break
        t = time.perf_counter()
        uv, ub = unrolled_grad(k)
        torch.cuda.synchronize()
        unrolled[k] = {"iterations": k, "ms": (time.perf_counter() - t) * 1e3,
                       "max_rel_diff_values_grad": rel(uv, gv), "max_rel_diff_b_grad": rel(ub, gb),
                       "error_values_grad": rel(uv, gv_ref), "error_b_grad": rel(ub, gb_ref),
                       "peak_bytes": int(torch.cuda.max_memory_allocated() - base)}
        del uv, ub
        if unrolled[k]["error_values_grad"] <= err_adj["values"] and unrolled[k]["error_b_grad"] <= err_adj["b"]:
            matched = k
            break
    M.close()
    same, last = unrolled[iters], unrolled[max(unrolled)]
    ref = unrolled[matched] if matched else last
    return {"workload": "varcoef7_96", "n": int(A.n), "nnz": int(A.nnz), "forward_iterations": iters,
            "adjoint_gradients_per_s": 1.0 / t_adj, "adjoint_ms": t_adj * 1e3,
            "equal_accuracy": {"criterion": "each unrolled gradient at most as far (max relative difference) "
                                            "from the gradients of solves to ref_tol as the adjoint's",
                               "ref_tol": ref_tol,
                               "adjoint_error_values_grad": err_adj["values"], "adjoint_error_b_grad": err_adj["b"],
                               "reached_at_iterations": matched, "searched_iterations": sorted(unrolled),
                               "note": None if matched else "not reached: the speedup is against the most "
                                       "iterations run, a lower bound on the unrolled cost at equal accuracy"},
            "unrolled_autograd_gradients_per_s": 1e3 / ref["ms"], "speedup": ref["ms"] * 1e-3 / t_adj,
            "unrolled": [unrolled[k] for k in sorted(unrolled)],
            "speedup_vs_same_iterations": same["ms"] * 1e-3 / t_adj}


def suite(torch, prcg, problems):
    """Per-iteration time of every variant on every workload (printed, one
    JSON line per workload and kernel structure; the default structure's
    lines also give each kernel's time per launch)."""
    def shard():
        # one GPU's rows of the 128^3 problem split into 8 z-slabs (no halo)
        A = problems.poisson3d(128, 128, 16)
        return problems.Problem(name="poisson3d_128x128x16_jacobi", A=A, b=problems.uniform_vector(A.n, 2),
                                precond="jacobi")

    work = [("poisson2d_64", problems.config1, "none", 1e-10, 5000),
            ("poisson3d_128_jacobi", problems.config2, "jacobi", 1e-10, 1000),
            ("poisson3d_128x128x16_jacobi", shard, "jacobi", 1e-10, 2000),
            ("model_diag_1e6", problems.config3a, "none", 1e-10, 20000),
            ("varcoef27_160", problems.config3b, "none", 1e-10, 20000),
            ("varcoef7_96", problems.config5, "none", 1e-10, 20000)]
    for name, fn, pre, tol, maxit in work:
        pr = fn()
        M = prcg.Matrix(pr.A.row_ptr, pr.A.col_idx, pr.A.values, pre)
        b = torch.as_tensor(pr.b, device="cuda")
        for kern in STRUCTURES:
            M.set_kernels(kern)
            out = {"workload": name, "n": pr.A.n, "nnz": pr.A.nnz, "kernels": kern}
            for v in variants_of(kern):
                x, info = M.solve(b, v, tol, maxit)
                best = float("inf")
                for _ in range(2):
                    torch.cuda.synchronize()
                    t = time.perf_counter()
                    x, info = M.solve(b, v, tol, maxit)
                    torch.cuda.synchronize()
                    best = min(best, time.perf_counter() - t)
                out[v] = {"iters": info.iters, "status": info.status, "relres_true": info.relres_true,
                          "us_per_iter": best / max(info.iters, 1) * 1e6, "solve_ms": best * 1e3}
                if kern == "auto":
                    # each kernel of the default structure, 20 launches timed with HIP events
                    out[v]["kernels_us"] = {k: ms * 1e3 for k, ms in M.time_kernels(v, 20)}
            print(json.dumps(out), flush=True)
        M.close()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch

    from paper_1905_01549_amd import prcg, problems, traffic

    torch.cuda.set_device(0)
    if args.suite:
        suite(torch, prcg, problems)
        return
    if args.batched_only:
        calibration_copy(torch)
        print(json.dumps(batched_section(torch, prcg, problems, traffic, args.batched_reps, not args.no_sequential,
                                         args.batched_config, args.batched_fusion)),
              flush=True)
        return
    if args.kernels_only and args.workload == "varcoef27_160":
        pr, workload, pre = problems.config3b(), "varcoef27_160", "none"
    else:
        pr, workload, pre = problems.config2(m=args.m), f"poisson3d_{args.m}_jacobi", "jacobi"
    A = pr.A
    M = prcg.Matrix(A.row_ptr, A.col_idx, A.values, pre)
    if args.grid:
        M.set_grid(args.grid)
    M.set_kernels(args.kernels)
    b = torch.as_tensor(pr.b, device="cuda")
    props = M.props
    n = A.n

    if args.kernels_only:
        calibration_copy(torch)
        kt = M.time_kernels(args.variant, 200)
        fused = any("fused" in name for name, _ in kt)  # the structure the variant runs
        jac = pre == "jacobi"
        kb = traffic.kernel_bytes(args.variant, jac, n, props.matrix_bytes, fused, nu_in_update=nu_split(M))
        kc = traffic.kernel_bytes(args.variant, jac, n, traffic.csr_matrix_bytes(n, A.nnz), fused,
                                  nu_in_update=nu_split(M))
        print(json.dumps({"workload": workload, "variant": args.variant, "launches": 200,
                          "kernels": {k: {"us": ms * 1e3, **(roofline_of(ms * 1e3, kb[k], kc[k]) if k in kb else {})}
                                      for k, ms in kt}}))
        return

    def solve(variant):
        x, info = M.solve(b, variant, TOL, MAXIT)
        assert info.status == "ok", info
        return info

    # flagship variant: warmup, then exactly `steps` timed solves
    for _ in range(args.warmup):
        solve(args.variant)
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    total_iters = 0
    t0 = time.perf_counter()
    start.record()
    for _ in range(args.steps):
        info = solve(args.variant)
        total_iters += info.iters
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_s = start.elapsed_time(end) / 1e3
    elapsed = max(wall, gpu_s)
    iters_per_s = total_iters / elapsed
    flagship = info

    # every variant under every kernel structure, same workload (best of 2 solves)
    variants = {}
    for kern in STRUCTURES:
        M.set_kernels(kern)
        for v in variants_of(kern):
            vi = solve(v)
            best = float("inf")
            for _ in range(2):
                torch.cuda.synchronize()
                t = time.perf_counter()
                vi = solve(v)
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t)
            kt = M.time_kernels(v, 50)
            fz = any("fused" in name for name, _ in kt)  # the structure this variant ran
            it_bytes = traffic.iteration_bytes(v, True, n, props.matrix_bytes, fz, kern == "textbook", nu_split(M))
            kb = traffic.kernel_bytes(v, True, n, props.matrix_bytes, fz, kern == "textbook", nu_split(M))
            variants[f"{v}/{kern}"] = {
                "iters": vi.iters,
                "relres_true": vi.relres_true,
                "solve_ms": best * 1e3,
                "us_per_iter": best / vi.iters * 1e6,
                "iters_per_s": vi.iters / best,
                "algorithmic_GBps": it_bytes / (best / vi.iters) / 1e9,
                "bytes_per_iter": it_bytes,
                "kernels": {name: {"us": ms * 1e3, "GBps": kb.get(name, 0) / (ms * 1e-3) / 1e9} for name, ms in kt},
            }
    M.set_kernels(args.kernels)

    # dominant kernel of the flagship variant: the SpMV + inner-product kernel
    kt = dict(M.time_kernels(args.variant, 200))
    fused = any("fused" in name for name in kt)  # the structure the variant runs
    kb = traffic.kernel_bytes(args.variant, True, n, props.matrix_bytes, fused, nu_in_update=nu_split(M))
    dom = max((k for k in kt if k in kb), key=lambda k: kt[k])
    kc = traffic.kernel_bytes(args.variant, True, n, traffic.csr_matrix_bytes(n, A.nnz), fused,
                              nu_in_update=nu_split(M))
    rl = roofline_of(kt[dom] * 1e3, kb[dom], kc[dom])
    tb = load_traffic(dom, workload)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": rl["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": rl["frac"], "traffic": tb, "bytes": "sell64_format",
                "bytes_per_launch": kb[dom], "us_per_launch": kt[dom] * 1e3, "launches_timed": 200,
                "bytes_per_launch_csr_model": kc[dom], "achieved_csr_model": rl["achieved_csr_model"],
                "frac_csr_model": rl["frac_csr_model"]}

    cpu = None
    cpu_host = None
    if not args.no_cpu_baseline:
        # the oracle as it stands: complete PR-CG solves of the same workload
        # to 1e-10, repeated until about 10 s of CPU time have been spent
        import oracle
        done_iters, solves = 0, 0
        t = time.perf_counter()
        while solves == 0 or time.perf_counter() - t < args.cpu_seconds:
            ref = oracle.solve(A.row_ptr, A.col_idx, A.values, pr.b, args.variant, "jacobi", TOL, MAXIT)
            done_iters += ref["iters"]
            solves += 1
        dt = time.perf_counter() - t
        threads = oracle.max_threads()
        cpu = {"value": done_iters / dt, "unit": "CG iterations/s", "cores": threads,
               "kind": "oracle",
               "sample": f"{solves} complete {args.variant} solves to 1e-10 ({done_iters} iterations, {dt:.1f} s) "
                         f"of the same {workload} workload by the FP64 C oracle"}
        # the same oracle on one core: 40 iterations (a bounded sample of the solve)
        oracle.set_threads(1)
        t = time.perf_counter()
        one = oracle.solve(A.row_ptr, A.col_idx, A.values, pr.b, args.variant, "jacobi", 0.0, 40)
        dt1 = time.perf_counter() - t
        oracle.set_threads(threads)
        cpu_host = {"model": cpu_model(), "nproc": os.cpu_count(), "threads": threads,
                    "iters_per_s_all_threads": done_iters / dt,
                    "iters_per_s_one_thread": one["iters"] / dt1,
                    "one_thread_sample": f"{one['iters']} iterations from x0 = 0 ({dt1:.1f} s, incl. setup)"}

    triad = stream_triad(torch)
    # the HBM-bound 27-point workload first, on a device whose memory the
    # later sections have not fragmented (the adjoint's unrolled autograd
    # holds up to ~150 GB in torch's cache)
    varcoef27 = None if args.no_27pt else varcoef27_section(torch, prcg, problems, traffic)
    torch.cuda.empty_cache()
    batched = None if args.no_batched else batched_section(torch, prcg, problems, traffic)
    torch.cuda.empty_cache()
    adjoint = None if args.no_adjoint else adjoint_section(torch, prcg, problems)

    out = {
        "metric": "CG iterations/sec (FP64 PR-CG solve to 1e-10 relative residual)",
        "value": iters_per_s,
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload, "n": n, "nnz": A.nnz, "precond": "jacobi", "variant": args.variant,
                   "tol": TOL, "iters_per_solve": flagship.iters, "relres_true": flagship.relres_true,
                   "kernels": args.kernels, "format": "sell64" if props.format == 0 else
                   f"csr{props.lanes_per_row}", "grid": props.grid, "parallelism": "single GPU"},
        "hbm_GBps_algorithmic": variants[f"{args.variant}/{args.kernels}"]["algorithmic_GBps"],
        "hbm_frac": variants[f"{args.variant}/{args.kernels}"]["algorithmic_GBps"] / HBM_PEAK_GBS,
        "stream_triad_GBps": triad,
        "device": device_facts(torch),
        "frac_of_stream_triad": {"iteration": variants[f"{args.variant}/{args.kernels}"]["algorithmic_GBps"] / triad,
                                 roofline["kernel"]: roofline["achieved"] / triad},
        "variants": variants,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "cpu_host": cpu_host,
        "batched": batched,
        "adjoint": adjoint,
        "varcoef27_160": varcoef27,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
