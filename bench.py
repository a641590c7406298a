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
TOL = 1e-10
MAXIT = 1000


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--variant", default="pr")
    ap.add_argument("--grid", type=int, default=0, help="override the workgroup count (tuning)")
    ap.add_argument("--kernels", default="two_pass", help="kernel structure of the flagship run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=40)
    ap.add_argument("--m", type=int, default=128, help="grid edge (128 = the benchmark workload)")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only time the flagship variant's kernels (the launches the roofline uses)")
    return ap.parse_args()


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1905_01549_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
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


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch

    from paper_1905_01549_amd import prcg, problems, traffic

    torch.cuda.set_device(0)
    pr = problems.config2(m=args.m)
    A = pr.A
    workload = f"poisson3d_{args.m}_jacobi"
    M = prcg.Matrix(A.row_ptr, A.col_idx, A.values, "jacobi")
    if args.grid:
        M.set_grid(args.grid)
    M.set_kernels(args.kernels)
    b = torch.as_tensor(pr.b, device="cuda")
    props = M.props
    n = A.n
    fused = args.kernels == "fused"

    if args.kernels_only:
        # a plain copy of known size (256 MiB read + 256 MiB written) to
        # calibrate hardware byte counters against
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        kt = M.time_kernels(args.variant, 200)
        kb = traffic.kernel_bytes(args.variant, True, n, props.matrix_bytes, fused)
        print(json.dumps({"workload": workload, "variant": args.variant, "launches": 200,
                          "kernels": {k: {"us": ms * 1e3, "bytes": kb.get(k, 0),
                                          "GBps": kb.get(k, 0) / (ms * 1e-3) / 1e9} for k, ms in kt}}))
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

    # every variant under both kernel structures, same workload (best of 2 solves)
    variants = {}
    for kern in ("two_pass", "fused", "textbook"):
        M.set_kernels(kern)
        for v in (("hs",) if kern == "textbook" else ("hs", "pr", "pipe_pr")):
            vi = solve(v)
            best = float("inf")
            for _ in range(2):
                torch.cuda.synchronize()
                t = time.perf_counter()
                vi = solve(v)
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t)
            fz = kern == "fused"
            it_bytes = traffic.iteration_bytes(v, True, n, props.matrix_bytes, fz, kern == "textbook")
            kt = M.time_kernels(v, 50)
            kb = traffic.kernel_bytes(v, True, n, props.matrix_bytes, fz, kern == "textbook")
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
    kb = traffic.kernel_bytes(args.variant, True, n, props.matrix_bytes, fused)
    dom = max((k for k in kt if k in kb), key=lambda k: kt[k])
    achieved = kb[dom] / (kt[dom] * 1e-3) / 1e9
    tb = load_traffic(dom, workload)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "bytes_per_launch": kb[dom], "us_per_launch": kt[dom] * 1e3,
                "traffic": tb}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        t = time.perf_counter()
        oracle.solve(A.row_ptr, A.col_idx, A.values, pr.b, args.variant, "jacobi", 0.0, args.cpu_iters)
        dt = time.perf_counter() - t
        cpu = {"value": args.cpu_iters / dt, "unit": "CG iterations/s", "cores": oracle.max_threads(),
               "kind": "oracle",
               "sample": f"{args.cpu_iters} PR-CG iterations (with initialisation) of the same "
                         f"{workload} workload, FP64 C oracle"}

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
        "variants": variants,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
