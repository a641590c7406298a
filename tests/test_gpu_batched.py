"""GPU parity of the batched solver (persistent and lockstep modes) against
the oracle, system by system: at the GPU's iteration count the solution
matches the oracle to 1e-10 relative, the stopping iteration agrees to +-1
and the status agrees."""
import numpy as np
import pytest

import oracle
from paper_1905_01549_amd import problems as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def prcg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1905_01549_amd import prcg as mod
    mod.load_library()
    return mod


def small_batch(nsys=12, nmin=64, nmax=3000):
    mats, bs = [], []
    for s in range(nsys):
        A, b, xs, eps = P.batch_system(s, nmin, nmax)
        mats.append(A)
        bs.append(b)
    A, offs = P.block_diag(mats)
    return A, offs, np.concatenate(bs), mats, bs


def check_systems(x, iters, status, mats, bs, offs, variant, precond, tol, which=None):
    which = range(len(mats)) if which is None else which
    for s in which:
        A, b = mats[s], bs[s]
        xs = x[offs[s]:offs[s + 1]]
        ref_stop = oracle.solve(A.row_ptr, A.col_idx, A.values, b, variant, precond, tol, 20000)
        assert status[s] == ref_stop["status"], (s, status[s], ref_stop["status"])
        assert abs(int(iters[s]) - ref_stop["iters"]) <= 1, (s, iters[s], ref_stop["iters"])
        ref = oracle.solve(A.row_ptr, A.col_idx, A.values, b, variant, precond, 0.0, int(iters[s]))
        assert np.linalg.norm(xs - ref["x"]) <= 1e-10 * np.linalg.norm(ref["x"]), s


@pytest.mark.parametrize("precond", ["none", "jacobi"])
@pytest.mark.parametrize("variant", ["pr", "hs", "pipe_pr", "m", "pipe_m"])
def test_batched_matches_oracle(prcg, variant, precond):
    A, offs, b, mats, bs = small_batch()
    M = prcg.Matrix(A.row_ptr, A.col_idx, A.values, precond)
    B = prcg.Batch(M, offs)
    x, iters, status = B.solve(b, variant, 1e-10, 5000)
    check_systems(x.cpu().numpy(), iters, status, mats, bs, offs, variant, precond, 1e-10)
    nt, grid = B.config(variant)
    assert nt in (256, 512, 1024) and grid >= 1


@pytest.mark.parametrize("config", ["512,2", "1024,1"])
@pytest.mark.parametrize("variant", ["pr", "pipe_pr", "hs"])
def test_packed_and_mixed_slices(prcg, variant, config, monkeypatch):
    """Systems whose slices are packed (explicit columns, rows of different
    lengths) next to stencil systems (offset-aligned slices, paired in the
    product), and tiny systems of fewer slices than wavefronts: each system
    against the oracle."""
    monkeypatch.setenv("PRCG_BATCH_CONFIG", config)
    mats = [P.random_spd(700 + 173 * s, 5.0, 20 + s) for s in range(3)]
    mats += [P.batch_system(s, 64, 3000)[0] for s in range(3)]
    mats += [P.poisson2d(3), P.random_spd(40, 3.0, 9)]
    bs = [P.uniform_vector(A.n, 30 + s) for s, A in enumerate(mats)]
    A, offs = P.block_diag(mats)
    M = prcg.Matrix(A.row_ptr, A.col_idx, A.values, "jacobi")
    B = prcg.Batch(M, offs)
    x, iters, status = B.solve(np.concatenate(bs), variant, 1e-10, 5000)
    check_systems(x.cpu().numpy(), iters, status, mats, bs, offs, variant, "jacobi", 1e-10)


@pytest.mark.parametrize("config", ["256,1", "512,2", "1024,1"])
def test_every_workgroup_size(prcg, config, monkeypatch):
    monkeypatch.setenv("PRCG_BATCH_CONFIG", config)
    A, offs, b, mats, bs = small_batch(9)
    M = prcg.Matrix(A.row_ptr, A.col_idx, A.values, "none")
    B = prcg.Batch(M, offs)
    x, iters, status = B.solve(b, "pr", 1e-10, 5000)
    assert B.config("pr")[0] == int(config.split(",")[0])
    check_systems(x.cpu().numpy(), iters, status, mats, bs, offs, "pr", "none", 1e-10)


def test_batched_is_repeatable_and_x0_is_used(prcg, monkeypatch):
    monkeypatch.setenv("PRCG_BATCH_CONFIG", "512,2")
    A, offs, b, mats, bs = small_batch(7)
    M = prcg.Matrix(A.row_ptr, A.col_idx, A.values, "jacobi")
    B = prcg.Batch(M, offs)
    x1, i1, _ = B.solve(b, "pipe_pr", 1e-10, 5000)
    x2, i2, _ = B.solve(b, "pipe_pr", 1e-10, 5000)
    assert np.array_equal(x1.cpu().numpy(), x2.cpu().numpy()) and np.array_equal(i1, i2)
    # starting from the solution: every system converges at k = 0
    x3, i3, s3 = B.solve(b, "pr", 1e-6, 5000, x0=x1)
    assert np.all(i3 == 0) and all(st == "ok" for st in s3)


def test_zero_block_and_maxit(prcg, monkeypatch):
    monkeypatch.setenv("PRCG_BATCH_CONFIG", "256,2")
    A, offs, b, mats, bs = small_batch(5)
    b = b.copy()
    b[offs[2]:offs[3]] = 0.0
    M = prcg.Matrix(A.row_ptr, A.col_idx, A.values, "none")
    B = prcg.Batch(M, offs)
    x, iters, status = B.solve(b, "pr", 1e-10, 5000, x0=np.ones(A.n))
    x = x.cpu().numpy()
    assert iters[2] == 0 and status[2] == "ok" and np.all(x[offs[2]:offs[3]] == 0.0)
    x, iters, status = B.solve(b, "hs", 0.0, 7)
    assert all(int(k) == 7 for s, k in enumerate(iters) if s != 2)
    assert all(st == "not_converged" for s, st in enumerate(status) if s != 2)


@pytest.mark.parametrize("precond", ["none", "jacobi"])
@pytest.mark.parametrize("variant", ["pr", "m"])
def test_lockstep_matches_oracle(prcg, variant, precond):
    A, offs, b, mats, bs = small_batch()
    M = prcg.Matrix(A.row_ptr, A.col_idx, A.values, precond)
    B = prcg.Batch(M, offs)
    B.set_mode("lockstep")
    x, iters, status = B.solve(b, variant, 1e-10, 5000)
    assert B.mode(variant) == "lockstep"
    check_systems(x.cpu().numpy(), iters, status, mats, bs, offs, variant, precond, 1e-10)


def test_lockstep_packed_tiny_and_ragged_groups(prcg):
    """Packed slices next to offset-aligned ones, systems of one to five
    slices (row groups of one to four slices, partial last slices) in
    lockstep: each system against the oracle."""
    mats = [P.random_spd(700 + 173 * s, 5.0, 20 + s) for s in range(3)]
    mats += [P.batch_system(s, 64, 3000)[0] for s in range(3)]
    mats += [P.poisson2d(3), P.random_spd(40, 3.0, 9), P.poisson2d(16, 20)]
    bs = [P.uniform_vector(A.n, 30 + s) for s, A in enumerate(mats)]
    A, offs = P.block_diag(mats)
    M = prcg.Matrix(A.row_ptr, A.col_idx, A.values, "jacobi")
    B = prcg.Batch(M, offs)
    B.set_mode("lockstep")
    x, iters, status = B.solve(np.concatenate(bs), "pr", 1e-10, 5000)
    check_systems(x.cpu().numpy(), iters, status, mats, bs, offs, "pr", "jacobi", 1e-10)


def test_lockstep_zero_block_maxit_x0_and_repeatability(prcg):
    A, offs, b, mats, bs = small_batch(5)
    b = b.copy()
    b[offs[2]:offs[3]] = 0.0
    M = prcg.Matrix(A.row_ptr, A.col_idx, A.values, "none")
    B = prcg.Batch(M, offs)
    B.set_mode("lockstep")
    x, iters, status = B.solve(b, "pr", 1e-10, 5000, x0=np.ones(A.n))
    x = x.cpu().numpy()
    assert iters[2] == 0 and status[2] == "ok" and np.all(x[offs[2]:offs[3]] == 0.0)
    x2, iters2, _ = B.solve(b, "pr", 1e-10, 5000, x0=np.ones(A.n))
    assert np.array_equal(x, x2.cpu().numpy()) and np.array_equal(iters, iters2)
    x, iters, status = B.solve(b, "pr", 0.0, 7)  # not a multiple of the 16-iteration chunk
    assert all(int(k) == 7 for s, k in enumerate(iters) if s != 2)
    assert all(st == "not_converged" for s, st in enumerate(status) if s != 2)
    x, iters, status = B.solve(b, "pr", 0.0, 0)
    assert np.all(iters == 0)
    xs, _, _ = B.solve(b, "pr", 1e-10, 5000)
    x, iters, status = B.solve(b, "pr", 1e-6, 5000, x0=xs)
    assert np.all(iters == 0) and all(st == "ok" for st in status)


def test_mode_selection(prcg):
    A, offs, b, mats, bs = small_batch(4)
    M = prcg.Matrix(A.row_ptr, A.col_idx, A.values, "none")
    B = prcg.Batch(M, offs)
    assert B.mode("pr") is None
    B.solve(b, "pr", 1e-10, 5000)
    assert B.mode("pr") in ("persistent", "lockstep") and B.mode("m") == B.mode("pr")
    B.set_mode("lockstep")
    assert B.mode("pr") is None
    B.solve(b, "hs", 1e-10, 5000)
    assert B.mode("hs") == "persistent"  # HS-CG has no lockstep mode
    with pytest.raises(prcg.PrcgError):
        prcg.prcg_batch_set_mode(B.handle, 3)


def test_block_structure_is_checked(prcg):
    A, offs, b, mats, bs = small_batch(3)
    M = prcg.Matrix(A.row_ptr, A.col_idx, A.values, "none")
    bad = offs.copy()
    bad[1] += 5  # splits a system: its couplings now cross a block boundary
    with pytest.raises(prcg.PrcgError):
        prcg.Batch(M, bad)
    with pytest.raises(prcg.PrcgError):
        prcg.Batch(M, offs[::-1].copy())


@pytest.fixture(scope="module")
def batch512():
    return P.config4()


@pytest.mark.parametrize("mode,fusion,precond", [("persistent", "auto", "none"), ("lockstep", "off", "none"),
                                                 ("lockstep", "on", "none"), ("lockstep", "on", "jacobi")])
def test_full_batched_workload_sampled(prcg, batch512, mode, fusion, precond):
    """All 512 systems (n from 1k to 64k) in one solve; the oracle checks the
    largest, the smallest and two more systems; every system's true residual
    is checked on the host."""
    A, offs, b, xstar, eps = batch512
    M = prcg.Matrix(A.row_ptr, A.col_idx, A.values, precond)
    B = prcg.Batch(M, offs)
    B.set_mode(mode)
    B.set_fusion(fusion)
    x, iters, status = B.solve(b, "pr", 1e-10, 20000)
    assert B.mode("pr") == mode
    if mode == "lockstep":
        assert B.props("pr")["fused"] == (fusion == "on")
    x = x.cpu().numpy()
    assert all(st == "ok" for st in status)
    sizes = np.diff(offs)
    sample = sorted({int(np.argmax(sizes)), int(np.argmin(sizes)), 17, 300})
    mats = {s: P.batch_system(s)[0] for s in sample}
    for s in sample:
        As = mats[s]
        bsys = b[offs[s]:offs[s + 1]]
        ref = oracle.solve(As.row_ptr, As.col_idx, As.values, bsys, "pr", precond, 0.0, int(iters[s]))
        xs = x[offs[s]:offs[s + 1]]
        assert np.linalg.norm(xs - ref["x"]) <= 1e-10 * np.linalg.norm(ref["x"]), s
    S = A.scipy()
    res = S @ x - b
    for s in range(len(sizes)):
        sl = slice(offs[s], offs[s + 1])
        assert np.linalg.norm(res[sl]) <= 2e-10 * np.linalg.norm(b[sl]), s


@pytest.mark.parametrize("mode,config", [("persistent", "256,1"), ("persistent", "512,2"), ("lockstep", "off"),
                                         ("lockstep", "on")])
def test_nan_system_leaves_neighbours_alone(prcg, mode, config, monkeypatch):
    """A system whose right-hand side holds NaN breaks down on its own: the
    zero slots of its neighbours' boundary rows read only their own system's
    vectors, so every other system still matches the oracle."""
    if mode == "persistent":
        monkeypatch.setenv("PRCG_BATCH_CONFIG", config)
    A, offs, b, mats, bs = small_batch(6)
    b = b.copy()
    bad = 2
    b[offs[bad]] = np.nan          # first row: read by the previous system's last rows
    b[offs[bad + 1] - 1] = np.nan  # last row: read by the next system's first rows
    bs = list(bs)
    bs[bad] = b[offs[bad]:offs[bad + 1]].copy()
    M = prcg.Matrix(A.row_ptr, A.col_idx, A.values, "none")
    B = prcg.Batch(M, offs)
    B.set_mode(mode)
    if mode == "lockstep":
        B.set_fusion(config)  # fused: the recomputed p' of the window reads the NaN system's rows only
    x, iters, status = B.solve(b, "pr", 1e-10, 5000)
    x = x.cpu().numpy()
    ref = oracle.solve(mats[bad].row_ptr, mats[bad].col_idx, mats[bad].values, bs[bad], "pr", "none", 1e-10, 5000)
    assert status[bad] == ref["status"] == "breakdown", (status[bad], ref["status"])
    others = [s for s in range(len(mats)) if s != bad]
    check_systems(x, iters, status, mats, bs, offs, "pr", "none", 1e-10, which=others)
    assert all(np.all(np.isfinite(x[offs[s]:offs[s + 1]])) for s in others)


@pytest.mark.parametrize("threads,per_cu,q", [(256, 1, 1), (256, 8, 2), (512, 4, 1), (1024, 2, 2)])
def test_every_persistent_candidate(prcg, threads, per_cu, q):
    """Each launch shape the autotuner may pick (threads per workgroup x
    workgroups per compute unit x slices multiplied together per wavefront),
    fixed through prcg_batch_set_config: every system against the oracle."""
    A, offs, b, mats, bs = small_batch(9)
    M = prcg.Matrix(A.row_ptr, A.col_idx, A.values, "jacobi")
    B = prcg.Batch(M, offs)
    B.set_config(threads, per_cu, q, 0)
    B.set_mode("persistent")
    x, iters, status = B.solve(b, "pr", 1e-10, 5000)
    p = B.props("pr")
    assert (p["threads"], p["slices_in_flight"], p["mode"]) == (threads, q, "persistent")
    check_systems(x.cpu().numpy(), iters, status, mats, bs, offs, "pr", "jacobi", 1e-10)


def test_slices_in_flight_do_not_change_the_bits(prcg):
    """Multiplying one or two slices per wavefront at a time feeds the rows
    to the sums in the same order: identical results."""
    A, offs, b, mats, bs = small_batch(7)
    M = prcg.Matrix(A.row_ptr, A.col_idx, A.values, "none")
    out = []
    for q in (1, 2):
        B = prcg.Batch(M, offs)
        B.set_config(512, 2, q, 0)
        B.set_mode("persistent")
        x, iters, _ = B.solve(b, "pipe_pr", 1e-10, 5000)
        out.append((x.cpu().numpy(), iters))
        B.close()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("group_slices", [8, 16, 32])
@pytest.mark.parametrize("precond", ["none", "jacobi"])
def test_every_lockstep_group_size(prcg, group_slices, precond):
    """Lockstep row groups of 8, 16 and 32 slices (2, 4, 8 per wavefront),
    stencil systems (uniform groups) next to packed and tiny ones: every
    system against the oracle."""
    mats = [P.random_spd(700 + 173 * s, 5.0, 20 + s) for s in range(2)]
    mats += [P.batch_system(s, 64, 5000)[0] for s in range(5)]
    mats += [P.poisson2d(3), P.poisson2d(40, 37)]
    bs = [P.uniform_vector(A.n, 50 + s) for s, A in enumerate(mats)]
    A, offs = P.block_diag(mats)
    M = prcg.Matrix(A.row_ptr, A.col_idx, A.values, precond)
    B = prcg.Batch(M, offs)
    B.set_config(0, 0, 0, group_slices)
    B.set_mode("lockstep")
    x, iters, status = B.solve(np.concatenate(bs), "pr", 1e-10, 5000)
    p = B.props("pr")
    assert p["group_slices"] == group_slices and p["mode"] == "lockstep"
    assert 0 < p["uniform_groups"] < p["groups"]
    check_systems(x.cpu().numpy(), iters, status, mats, bs, offs, "pr", precond, 1e-10)


def test_autotuned_configuration_is_reported(prcg):
    A, offs, b, mats, bs = small_batch(6)
    M = prcg.Matrix(A.row_ptr, A.col_idx, A.values, "none")
    B = prcg.Batch(M, offs)
    assert B.props("pr")["threads"] == 0 and B.props("pr")["mode"] is None
    x, iters, status = B.solve(b, "pr", 1e-10, 5000)
    p = B.props("pr")
    assert p["threads"] in (256, 512, 1024) and p["slices_in_flight"] in (1, 2) and p["grid"] >= 1
    assert p["group_slices"] in (8, 16, 32) and p["mode"] in ("persistent", "lockstep")
    assert p["nsys"] == 6 and p["n"] == A.n and p["matrix_bytes"] >= 8 * p["stored_entries"]
    check_systems(x.cpu().numpy(), iters, status, mats, bs, offs, "pr", "none", 1e-10)
    for bad in [(300, 0, 0, 0), (1024, 4, 0, 0), (0, 9, 0, 0), (0, 0, 3, 0), (0, 0, 0, 12)]:
        with pytest.raises(prcg.PrcgError):
            B.set_config(*bad)


def stencil_batch():
    """Systems whose row groups are all offset-aligned (2D 5-point stencils,
    anisotropic and not, whose boundary slices hold 3 or 4 slots, a 1D
    3-point system, a one-row system and a 2000 x 2 grid whose span of 4000
    rows needs a window eight times the group's rows): sizes from one row to
    about 6,000 rows, so groups end ragged and some systems hold one group."""
    mats = [P.batch_system(s, 64, 6000)[0] for s in range(9)]
    mats += [P.poisson2d(3), P.poisson2d(5, 7), P.aniso2d(40, 3, 0.01), P.poisson2d(70, 2), P.poisson2d(1, 1),
             P.poisson2d(50, 1), P.poisson2d(2000, 2)]
    bs = [P.uniform_vector(A.n, 70 + s) for s, A in enumerate(mats)]
    A, offs = P.block_diag(mats)
    return A, offs, np.concatenate(bs), mats, bs


@pytest.mark.parametrize("precond", ["none", "jacobi"])
@pytest.mark.parametrize("group_slices", [8, 16])
@pytest.mark.parametrize("variant", ["pr", "m"])
def test_fused_lockstep_equals_three_launches(prcg, group_slices, variant, precond):
    """The fused lockstep iteration (update and product in one launch, p'
    recomputed past the group's edges) gives the bits of three launches per
    iteration, with and without Jacobi: from x0 = 0 to convergence, from
    x0 != 0, and for a maxit that is not a multiple of the 16-iteration
    chunk; every system of the fused run against the oracle."""
    A, offs, b, mats, bs = stencil_batch()
    M = prcg.Matrix(A.row_ptr, A.col_idx, A.values, precond)
    x0 = P.uniform_vector(A.n, 99)
    runs = {}
    for fusion in ("off", "on"):
        B = prcg.Batch(M, offs)
        B.set_config(0, 0, 0, group_slices)
        B.set_mode("lockstep")
        B.set_fusion(fusion)
        out = [B.solve(b, variant, 1e-10, 5000), B.solve(b, variant, 1e-10, 5000, x0=x0),
               B.solve(b, variant, 0.0, 23)]
        p = B.props(variant)
        assert p["fused"] == (fusion == "on") and p["group_slices"] == group_slices
        assert p["uniform_groups"] == p["groups"]
        runs[fusion] = [(x.cpu().numpy(), iters, status) for x, iters, status in out]
        B.close()
    for (xa, ia, sa), (xb, ib, sb) in zip(runs["off"], runs["on"]):
        assert np.array_equal(xa, xb) and np.array_equal(ia, ib) and sa == sb
    x, iters, status = runs["on"][0]
    check_systems(x, iters, status, mats, bs, offs, variant, precond, 1e-10)
    big = np.diff(offs) > 200  # the 9-row system terminates (exactly) sooner
    assert np.all(runs["on"][2][1][big] == 23) and np.all(runs["on"][2][1] <= 23)


def test_fusion_settings_are_checked(prcg):
    """The fused iteration needs uniform groups of a bounded span: asking
    for it elsewhere fails with PRCG_EINVAL at the solve, as does an unknown
    setting; 'auto' picks three launches there."""
    mixed = [P.random_spd(900, 5.0, 3), P.batch_system(0, 64, 3000)[0]]
    Am, offm = P.block_diag(mixed)
    Mm = prcg.Matrix(Am.row_ptr, Am.col_idx, Am.values, "none")
    Bm = prcg.Batch(Mm, offm)
    Bm.set_mode("lockstep")
    Bm.set_fusion("on")
    with pytest.raises(prcg.PrcgError):
        Bm.solve(P.uniform_vector(Am.n, 5), "pr", 1e-10, 5000)
    with pytest.raises(prcg.PrcgError):
        prcg.prcg_batch_set_fusion(Bm.handle, 3)
    # a stencil whose span (2 x 7000 rows) exceeds what the LDS window holds:
    # 'on' fails, 'auto' runs three launches and matches the oracle
    wide = [P.poisson2d(7000, 2), P.batch_system(1, 64, 3000)[0]]
    bw = [P.uniform_vector(A_.n, 40 + s) for s, A_ in enumerate(wide)]
    Aw, offw = P.block_diag(wide)
    Mw = prcg.Matrix(Aw.row_ptr, Aw.col_idx, Aw.values, "none")
    Bw = prcg.Batch(Mw, offw)
    Bw.set_mode("lockstep")
    Bw.set_fusion("on")
    with pytest.raises(prcg.PrcgError):
        Bw.solve(np.concatenate(bw), "pr", 1e-10, 5000)
    Bw.set_fusion("auto")
    x, iters, status = Bw.solve(np.concatenate(bw), "pr", 1e-10, 5000)
    assert Bw.props("pr")["fused"] == 0
    check_systems(x.cpu().numpy(), iters, status, wide, bw, offw, "pr", "none", 1e-10)
