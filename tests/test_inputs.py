"""The seeded synthetic workloads have the documented sizes and structure
(CPU): symmetric, positive diagonals, weak diagonal dominance (SPD for these
M-matrices and their variable-coefficient forms), reproducible from their
seeds."""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_1905_01549_amd import problems as P


def check_spd_structure(A, strict_rows=True):
    S = A.scipy()
    assert (S - S.T).count_nonzero() == 0 or abs(S - S.T).max() == 0.0
    d = S.diagonal()
    assert np.all(d > 0)
    off = np.asarray(abs(S).sum(axis=1)).ravel() - d
    assert np.all(d >= off * (1 - 1e-12))          # weakly diagonally dominant
    if strict_rows:
        assert np.any(d > off * (1 + 1e-12))       # and strictly on some row (irreducible: SPD)


@pytest.mark.parametrize("name, n, nnz", [
    ("config1", 4_096, 20_224),
    ("config2", 2_097_152, 14_581_760),
    ("config3a", 1_000_000, 1_000_000),
    ("config5", 884_736, 6_137_856),
])
def test_workload_sizes(name, n, nnz):
    pr = getattr(P, name)()
    assert (pr.A.n, pr.A.nnz) == (n, nnz)
    assert pr.b.shape == (n,) and np.all(np.isfinite(pr.b))


def test_stencils_are_spd_m_matrices():
    for A in (P.config1().A, P.poisson3d(12), P.varcoef27(10, 3), P.varcoef7(10, 5), P.aniso2d(9, 7, 1e-3)):
        check_spd_structure(A)


def test_model_spectrum_endpoints_and_order():
    """eq. model: lambda_1 = 1e-3, lambda_n = 1e3, non-decreasing (the first
    hundreds cluster at lambda_1), geometric weighting by rho."""
    lam = P.model_spectrum(1000, 1e-3, 1e3, 0.9)
    assert lam[0] == pytest.approx(1e-3) and lam[-1] == pytest.approx(1e3)
    assert np.all(np.diff(lam) >= 0) and lam[-1] / lam[-2] > 1.1
    i = np.arange(1, 1001)
    assert np.allclose(lam, 1e-3 + (i - 1) / 999 * (1e3 - 1e-3) * 0.9 ** (1000 - i), rtol=1e-14, atol=0)


def test_batched_workload_blocks():
    A, offs, b, xs, eps = P.config4()
    sizes = np.diff(offs)
    assert len(sizes) == 512 and A.n == offs[-1] == 17_399_581
    assert sizes.min() >= 900 and sizes.max() <= 66_000  # n ~ U{1k..64k}, rounded to a grid
    eps = np.asarray(eps)
    assert np.all((eps >= 1e-3) & (eps <= 1.0))
    # no coupling across systems
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    sys_of = np.searchsorted(offs, np.arange(A.n), side="right") - 1
    assert np.array_equal(sys_of[rows], sys_of[A.col_idx])


def test_generators_are_reproducible():
    a, b_ = P.varcoef27(8, 3), P.varcoef27(8, 3)
    assert np.array_equal(a.values, b_.values) and np.array_equal(a.col_idx, b_.col_idx)
    assert np.array_equal(P.uniform_vector(100, 7), P.uniform_vector(100, 7))
    assert not np.array_equal(P.uniform_vector(100, 7), P.uniform_vector(100, 8))
