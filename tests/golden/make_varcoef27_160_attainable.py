"""Writes varcoef27_160_attainable.json: the oracle's attainable accuracy on
the 27-point variable-coefficient problem at full size (160^3 cells,
n = 4,096,000, nnz = 109,215,352, lognormal(0,1) cell coefficients, x* ~
U[-1,1], b = A x*, no preconditioner, x0 = 0), for HS-CG, PR-CG and
pipe-PR-CG.

The oracle alone computes every stored number; the GPU tests compare their
own runs with them by the paper's criterion for attainable accuracy
(Section 4: agreement within 10% on a log scale).  Each variant runs
MAXIT iterations with tol = 0 and the true relative residual
||b - A x_k|| / ||b|| recorded at every k.

Run from the repository root:  python tests/golden/make_varcoef27_160_attainable.py
(about 6 minutes on 8 host cores).
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1905_01549_amd import problems  # noqa: E402

MAXIT = 2000
CHECKPOINTS = (1200, 1400, 1600, 1800, 2000)
TOL = 1e-10


def main():
    pr = problems.config3b()
    A = pr.A
    out = {
        "source": "oracle/prcg_oracle.c on problems.config3b() (written by this script; no GPU value enters)",
        "criterion": "Section 4: attainable accuracy compared within 10% on a log scale",
        "workload": "varcoef27_160", "n": int(A.n), "nnz": int(A.nnz), "maxit": MAXIT, "tol_stop": TOL,
        "checkpoints": list(CHECKPOINTS), "variants": {},
    }
    for v in ("hs", "pr", "pipe_pr"):
        ref = oracle.solve(A.row_ptr, A.col_idx, A.values, pr.b, v, "none", 0.0, MAXIT, diagnostics=["true_res"])
        h, t = ref["history"], ref["true_res"]
        stop = int(np.argmax(h <= TOL)) if np.any(h <= TOL) else None
        kmin = int(np.nanargmin(t))
        out["variants"][v] = {
            "iters": int(ref["iters"]),
            "stop_iteration_tol": stop,
            "true_res_at_stop": float(t[stop]) if stop is not None else None,
            "min_true_res": float(t[kmin]), "argmin_true_res": kmin,
            "true_res_at_checkpoints": {str(k): float(t[k]) for k in CHECKPOINTS},
            "updated_res_at_checkpoints": {str(k): float(h[k]) for k in CHECKPOINTS},
        }
        print(v, json.dumps(out["variants"][v]), flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "varcoef27_160_attainable.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
