"""Adjoint (gradient) checks on the GPU.

* 12^3 variable-coefficient 7-point instance: dL/db and dL/dA_e against a
  dense FP64 reference (numpy solves), max-norm relative error <= 1e-9.
* 96^3 instance (n = 884,736): central finite differences (h = 1e-6) of
  L = w^T A^{-1} b on 64 random symmetric pairs (A_ij and A_ji moved
  together, so A stays SPD; compared with g_ij + g_ji; diagonal entries
  alone), each perturbed solve done as a correction solve
  A_h d = b - A_h x^ to 1e-12 of its own right-hand side, so that the
  difference of the two losses is w^T (d+ - d-) and solver noise cancels.
"""
import numpy as np
import pytest

from paper_1905_01549_amd import problems as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("variant", ["pr", "pipe_pr", "hs"])
def test_dense_reference_gradient(torch_mod, variant):
    torch = torch_mod
    from paper_1905_01549_amd import prcg
    from paper_1905_01549_amd.autograd import solve

    A = P.varcoef7(12, 5)
    rng = np.random.default_rng(12)
    b = rng.uniform(-1, 1, A.n)
    w = rng.standard_normal(A.n)
    M = prcg.Matrix(A.row_ptr, A.col_idx, A.values)
    vals = torch.tensor(A.values, device="cuda", requires_grad=True)
    bt = torch.tensor(b, device="cuda", requires_grad=True)
    x = solve(vals, bt, M, variant, 1e-13, 5000)
    loss = (torch.tensor(w, device="cuda") * x).sum()
    loss.backward()
    Ad = A.dense()
    xr = np.linalg.solve(Ad, b)
    lam = np.linalg.solve(Ad.T, w)
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    g_ref = -lam[rows] * xr[A.col_idx]
    gv = vals.grad.cpu().numpy()
    gb = bt.grad.cpu().numpy()
    assert np.max(np.abs(gv - g_ref)) <= 1e-9 * np.max(np.abs(g_ref))
    assert np.max(np.abs(gb - lam)) <= 1e-9 * np.max(np.abs(lam))
    assert np.max(np.abs(x.detach().cpu().numpy() - xr)) <= 1e-9 * np.max(np.abs(xr))


def test_gradient_only_for_b(torch_mod):
    torch = torch_mod
    from paper_1905_01549_amd import prcg
    from paper_1905_01549_amd.autograd import solve

    A = P.poisson2d(20)
    M = prcg.Matrix(A.row_ptr, A.col_idx, A.values)
    vals = torch.tensor(A.values, device="cuda")
    bt = torch.ones(A.n, device="cuda", dtype=torch.float64, requires_grad=True)
    x = solve(vals, bt, M)
    (x * x).sum().backward()
    Ad = A.dense()
    xr = np.linalg.solve(Ad, np.ones(A.n))
    lam = np.linalg.solve(Ad, 2 * xr)
    assert np.max(np.abs(bt.grad.cpu().numpy() - lam)) <= 1e-8 * np.max(np.abs(lam))


def test_finite_differences_96(torch_mod):
    torch = torch_mod
    from paper_1905_01549_amd import prcg

    pr = P.config5()
    A = pr.A
    w = pr.extra["w"]
    M = prcg.Matrix(A.row_ptr, A.col_idx, A.values)
    bt = torch.tensor(pr.b, device="cuda")
    wt = torch.tensor(w, device="cuda")
    # forward solution polished to 1e-13 and its gradient
    x, info = M.solve(bt, "pr", 1e-13, 20000)
    assert info.status == "ok"
    gb, gv, ainfo = M.adjoint(x, wt, "pr", 1e-13, 20000)
    assert ainfo.status == "ok"
    g = gv.cpu().numpy()
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr)).astype(np.int64)
    cols = A.col_idx.astype(np.int64)
    # position of the transposed entry of every stored entry
    key = rows * A.n + cols
    tkey = cols * A.n + rows
    order = np.argsort(key)
    partner = order[np.searchsorted(key[order], tkey)]
    rng = np.random.default_rng(64)
    picks = rng.choice(A.nnz, 64, replace=False)
    h = 1e-6
    for e in picks:
        pe = partner[e]
        fd = []
        for sgn in (+1.0, -1.0):
            vals = A.values.copy()
            vals[e] += sgn * h
            if pe != e:
                vals[pe] += sgn * h
            M.set_values(vals)
            rh = bt - M.spmv(x)
            d, dinfo = M.solve(rh, "pr", 1e-12, 20000)
            assert dinfo.status == "ok"
            fd.append(float((wt * d).sum()))
        fdv = (fd[0] - fd[1]) / (2 * h)
        ana = g[e] + (g[pe] if pe != e else 0.0)
        assert abs(fdv - ana) <= 1e-5 * abs(ana) + 1e-12, (e, fdv, ana)
    M.set_values(A.values)
