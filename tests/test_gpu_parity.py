"""GPU path vs the CPU oracle, through the C ABI.

Every whole-solve case runs the oracle twice on the same seeded input, once
with sequential and once with blocked-pairwise reductions, and holds the GPU
to the band that pair fixes (parity_contract.check).  Kernel-level products
are held to a few ulps of the oracle's.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
import parity_contract as PC
from paper_2608_07327_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2608_07327_amd import mbpcg as M  # noqa: E402

DEV = torch.device("cuda:0")


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def check_against_oracle(A, b, s, tol=1e-8, jacobi=True, seed=0, U=None, max_iter=100000,
                         block_jacobi=0, floor=1e-10, tol_initial=0.0, profile=0):
    """One GPU solve against the oracle's two orderings, held to the FP64
    parity contract of parity_contract.check."""
    say("mbpcg", getattr(A, "n", None) or A.shape[0], "s", s, "seed", seed, "bj", block_jacobi,
        "tol0", tol_initial, "profile", profile)
    kw = dict(tol=tol, jacobi=jacobi, seed=seed, U=U, max_iter=max_iter,
              block_jacobi=block_jacobi, tol_initial=tol_initial)
    xo, io, xp, ip = PC.oracle_band(A, b, s, **kw)
    solver = M.Solver.from_matrix(A)
    Ud = None if U is None else dev(U)
    if block_jacobi:
        assert jacobi
        pre = dict(precond=M.PRECOND_BLOCK_JACOBI, block_size=block_jacobi)
    else:
        pre = dict(precond=M.PRECOND_JACOBI if jacobi else M.PRECOND_NONE)
    x, info = solver.solve(dev(b), s=s, tol=tol, seed=seed, U=Ud, max_iter=max_iter,
                           tol_initial=tol_initial, profile=profile, **pre)
    x = x.cpu().numpy()
    solver.close()
    PC.check(x, info, xo, io, xp, ip, tol, floor=floor, what=f"s={s} seed={seed}")
    return x, info, xo, io


# ------------------------------------------------------------- block product
@pytest.mark.parametrize("s", [1, 2, 4, 8, 16, 32])
def test_block_product_and_gram_small(s):
    A = W.diffusion3d(13)          # n = 2197: several tiles and a ragged tail
    say("block product", A.n, s)
    P = W.rng_for((70, s)).standard_normal((A.n, s))
    solver = M.Solver.from_matrix(A)
    Q = torch.empty((A.n, s), dtype=torch.float64, device=DEV)
    Cm = torch.zeros((s, s), dtype=torch.float64, device=DEV)
    solver.block_product(dev(P), Q, Cm, s, precond=M.PRECOND_JACOBI)
    d = np.sqrt(A.to_scipy().diagonal())
    As = W.CSR(A.n, A.rowptr, A.colind, A.vals / (d[np.repeat(np.arange(A.n), np.diff(A.rowptr))]
                                                   * d[A.colind]))
    Qo = O.matmul_block(As, P)
    Co = O.gram(P, Qo)
    Qg = Q.cpu().numpy()
    assert np.max(np.abs(Qg - Qo)) <= 1e-14 * np.max(np.abs(Qo)) * 8
    Cg = np.tril(Cm.cpu().numpy())
    assert np.max(np.abs(Cg - np.tril(Co))) <= 1e-12 * np.max(np.abs(Co))
    solver.close()


def _hub_laplacian():
    """Random graph Laplacian (avg degree 8, n = 3001) with node 0 joined to
    2500 others: its row and the tiles holding it need many LDS chunks."""
    import scipy.sparse as sp
    rng = W.rng_for((73,))
    L = W.graph_laplacian(3001, 8, 1e-2, rng).to_scipy().tolil()
    nb = rng.choice(np.arange(1, 3001), 2500, replace=False)
    for j in nb:
        if L[0, j] == 0:
            L[0, j] = L[j, 0] = -0.25
            L[0, 0] += 0.25
            L[j, j] += 0.25
    L = sp.csr_matrix(L)
    L.sort_indices()
    return W.CSR(L.shape[0], L.indptr.astype(np.int32), L.indices.astype(np.int32),
                 L.data.astype(np.float64))


@pytest.mark.parametrize("s", [1, 2, 4, 8, 16, 32])
def test_block_product_every_tile_shape(s):
    # every compiled (tile rows, lanes per row, columns per lane, loads in
    # flight), on the default grid and on an 8-workgroup grid, against the
    # oracle: two k-term sums in any order differ by at most 2 (k + 1) eps
    # (|A| |P|) per entry, and the Gram likewise over n terms
    A = _hub_laplacian()
    P = W.rng_for((74, s)).standard_normal((A.n, s))
    Qo = O.matmul_block(A, P)
    Co = O.gram(P, Qo)
    As = A.to_scipy()
    k = np.diff(A.rowptr)[:, None]
    eps = np.finfo(np.float64).eps
    bq = 2 * (k + 1) * eps * (abs(As) @ np.abs(P))
    bc = 2 * (A.n + 1) * eps * (np.abs(P).T @ np.abs(Qo)) + np.abs(P).T @ bq
    solver = M.Solver.from_matrix(A)
    Q = torch.empty((A.n, s), dtype=torch.float64, device=DEV)
    Cm = torch.zeros((s, s), dtype=torch.float64, device=DEV)
    Pd = dev(P)
    shapes = M.tile_shapes(s)
    assert shapes
    for sh in shapes:
        for wg in (0, 8):
            say("tile shape", s, sh, wg)
            solver.set_tile_shape(s, dict(sh, workgroups=wg))
            Q.fill_(np.nan)
            Cm.zero_()
            solver.block_product(Pd, Q, Cm, s, precond=M.PRECOND_NONE)
            Qg = Q.cpu().numpy()
            assert np.all(np.abs(Qg - Qo) <= bq), (sh, wg)
            Cg = np.tril(Cm.cpu().numpy())
            assert np.all(np.abs(Cg - np.tril(Co)) <= np.tril(bc)), (sh, wg)
    solver.close()


def test_set_tile_shape_rejects_unknown_shapes():
    A = W.poisson2d(16)
    solver = M.Solver.from_matrix(A)
    for bad in ({"tile_rows": 48, "lanes_per_row": 4, "cols_per_lane": 1, "loads_in_flight": 8},
                {"tile_rows": 64, "lanes_per_row": 3, "cols_per_lane": 1, "loads_in_flight": 8},
                {"tile_rows": 64, "lanes_per_row": 1, "cols_per_lane": 0, "loads_in_flight": 8}):
        with pytest.raises(M.MbpcgError):
            solver.set_tile_shape(4, bad)
    solver.close()


@pytest.mark.parametrize("s", [1, 4, 16, 32])
def test_dense_block_product(s):
    n = 300
    A = W.dense_spd(n, tag=(3, 40))
    say("dense block product", n, s)
    P = W.rng_for((71, s)).standard_normal((n, s))
    solver = M.Solver.from_matrix(A)
    Q = torch.empty((n, s), dtype=torch.float64, device=DEV)
    Cm = torch.zeros((s, s), dtype=torch.float64, device=DEV)
    solver.block_product(dev(P), Q, Cm, s, precond=M.PRECOND_NONE)
    Qo = O.matmul_block(A, P)
    assert np.max(np.abs(Q.cpu().numpy() - Qo)) <= 1e-13 * np.max(np.abs(Qo))
    Co = O.gram(P, Qo)
    assert np.max(np.abs(np.tril(Cm.cpu().numpy()) - np.tril(Co))) <= 1e-12 * np.abs(Co).max()
    solver.close()


def test_block_product_full_size_3d():
    # the 128^3 diffusion operator at s = 8: every row against the oracle
    A = W.diffusion3d(128)
    s = 8
    say("block product 128^3", s)
    P = W.rng_for((72,)).standard_normal((A.n, s))
    solver = M.Solver.from_matrix(A)
    Q = torch.empty((A.n, s), dtype=torch.float64, device=DEV)
    Cm = torch.zeros((s, s), dtype=torch.float64, device=DEV)
    solver.block_product(dev(P), Q, Cm, s, precond=M.PRECOND_NONE)
    Qo = O.matmul_block(A, P)
    assert np.max(np.abs(Q.cpu().numpy() - Qo)) <= 1e-13 * np.max(np.abs(Qo))
    Co = O.gram(P, Qo)
    assert np.max(np.abs(np.tril(Cm.cpu().numpy()) - np.tril(Co))) <= 1e-11 * np.abs(Co).max()
    solver.close()


# ------------------------------------------------------------ whole method
@pytest.mark.parametrize("s", [1, 2, 3, 4, 8])
def test_poisson2d_against_oracle(s):
    A = W.poisson2d(64)
    b = W.rhs(A.n, W.CFG_POISSON2D)
    check_against_oracle(A, b, s, seed=W.uniform_block_seed(1, s))


@pytest.mark.parametrize("s", [1, 4, 16])
def test_diffusion3d_against_oracle(s):
    A = W.diffusion3d(20)
    b = W.rhs(A.n, W.CFG_DIFFUSION3D)
    check_against_oracle(A, b, s, seed=W.uniform_block_seed(2, s))


@pytest.mark.parametrize("s", [5, 6, 7, 12, 24])
def test_padded_widths_against_oracle(s):
    # s below the padded block width S (8, 16, 32): the inactive columns
    # stay zero through the product, the Grams, the Cholesky QR and the
    # least squares
    A = W.diffusion3d(20)
    b = W.rhs(A.n, W.CFG_DIFFUSION3D)
    check_against_oracle(A, b, s, seed=W.uniform_block_seed(2, s))


@pytest.mark.parametrize("s", [5, 12, 20])
def test_padded_widths_dense_against_oracle(s):
    A = W.dense_spd(600, tag=(3, 41))
    b = W.rng_for((3, 42)).standard_normal(600)
    check_against_oracle(A, b, s, jacobi=False, seed=W.uniform_block_seed(3, s))


@pytest.mark.parametrize("s", [1, 4, 8, 16, 32])
def test_dense_against_oracle(s):
    # n = 600: two 256-row tiles and a ragged tail, two column ranges
    A = W.dense_spd(600, tag=(3, 41))
    b = W.rng_for((3, 42)).standard_normal(600)
    check_against_oracle(A, b, s, jacobi=False, seed=W.uniform_block_seed(3, s))


@pytest.mark.parametrize("s", [1, 4, 8])
def test_diffusion_with_inclusions_against_oracle(s):
    # highly conducting inclusions: a few isolated small eigenvalues of the
    # scaled operator (CG 158 iterations at n = 4096, s = 8 about 70)
    A = W.diffusion3d(16, inclusions=6, contrast=1e4, size=3)
    b = W.rhs(A.n, 81)
    check_against_oracle(A, b, s, seed=W.uniform_block_seed(81, s))


@pytest.mark.parametrize("kind", ["dense", "csr"])
@pytest.mark.parametrize("s", [2, 4, 8])
def test_near_singular_systems_against_oracle(kind, s):
    # kappa ~ 4e6 dense and a graph Laplacian shifted by 1e-6: the
    # termination's least squares on nearly dependent columns of B^
    if kind == "dense":
        A = W.dense_spd(256, tag=(W.CFG_DENSE, 95, 256), shift=1e-6)
        b = W.rng_for((96, 256)).standard_normal(256)
        jac = False
    else:
        A = W.graph_laplacian(2000, 8, 1e-6, W.rng_for((W.CFG_BATCH, 91, 2000, 6)))
        b = W.rng_for((93, 2000)).standard_normal(2000)
        jac = True
    x, info, xo, io = check_against_oracle(A, b, s, jacobi=jac, seed=W.uniform_block_seed(97, s))
    assert info["rel_res_true"] < 2e-8


@pytest.mark.parametrize("s", [4, 8, 16])
def test_ill_conditioned_dense_against_oracle(s):
    # A = G G^T / n + 1e-5 I, n = 2048 (kappa ~ 4e5): the combination's
    # coefficients are large, and the true-residual fallback decides
    n = 2048
    A = W.dense_spd(n, tag=(W.CFG_DENSE, 92, n), shift=1e-5)
    b = W.rng_for((93, 7)).standard_normal(n)
    x, info, xo, io = check_against_oracle(A, b, s, jacobi=False, seed=W.uniform_block_seed(94, s))
    t = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert abs(info["rel_res_true"] - t) <= 1e-3 * t, (t, info["rel_res_true"])


def test_true_residual_fallback_fires_as_in_the_oracle():
    # dense n = 512, shift 1e-5, s = 2: the combination passes the test on
    # B^ c but its true residual misses tol, and the best column's is lower;
    # both sides return the best column (used_fallback = 1)
    A = W.dense_spd(512, tag=(3, 512), shift=1e-5)
    b = W.rhs(512, (3, 512))
    x, info, xo, io = check_against_oracle(A, b, 2, jacobi=False, seed=0)
    assert io["used_fallback"] == 1 and io["rel_res_ls"] < 1e-8
    assert info["used_fallback"] == 1 and info["rel_res_true"] < 1e-8


# ------------------------------------------------- Alg. 1's two tolerances
@pytest.mark.parametrize("s", [1, 4, 8])
@pytest.mark.parametrize("profile", [0, 1])
def test_tol_initial_above_tol_against_oracle(s, profile):
    # the combination is tried from the iteration whose best column meets
    # tol_initial on, and ends the solve before the best column meets tol
    A = W.poisson2d(32)
    b = W.rhs(A.n, 41)
    x, info, xo, io = check_against_oracle(A, b, s, seed=3 + s, tol_initial=1e-6, profile=profile)
    assert info["status"] == 0


@pytest.mark.parametrize("tol0", [1e-5, 1e-9])
def test_tol_initial_on_diffusion_and_dense_against_oracle(tol0):
    A = W.diffusion3d(20)
    b = W.rhs(A.n, W.CFG_DIFFUSION3D)
    check_against_oracle(A, b, 4, seed=W.uniform_block_seed(2, 4), tol_initial=tol0)
    Ad = W.dense_spd(600, tag=(3, 41))
    bd = W.rng_for((3, 42)).standard_normal(600)
    check_against_oracle(Ad, bd, 8, jacobi=False, seed=W.uniform_block_seed(3, 8),
                         tol_initial=tol0)


def test_tol_initial_with_max_iter_between_the_tests():
    # capped while the combination is being tried: NOT_CONVERGED with the
    # best column, as in the oracle
    A = W.poisson2d(32)
    b = W.rhs(A.n, 41)
    x, info, xo, io = check_against_oracle(A, b, 4, seed=3, tol_initial=1e-6, max_iter=67)
    assert info["status"] == io["status"] == 1 and info["used_fallback"] == 1


# ------------------------------------------------------- block-Jacobi preconditioner
@pytest.mark.parametrize("s,bs", [(1, 8), (2, 4), (4, 8), (4, 32), (8, 16), (16, 8), (32, 4),
                                  (3, 16)])
def test_block_jacobi_against_oracle(s, bs):
    # 21^3 = 9261 rows: a ragged last block for every block size, several tiles
    A = W.diffusion3d(21)
    b = W.rhs(A.n, 71)
    _, info, _, io = check_against_oracle(A, b, s, seed=W.uniform_block_seed(71, s),
                                          block_jacobi=bs)
    assert info["status"] == 0


@pytest.mark.parametrize("s,bs", [(4, 8), (16, 32)])
def test_block_jacobi_dense_against_oracle(s, bs):
    A = W.dense_spd(600, tag=(3, 41))          # 600 rows: 600 % 32 = 24, ragged
    b = W.rng_for((3, 42)).standard_normal(600)
    check_against_oracle(A, b, s, seed=W.uniform_block_seed(72, s), block_jacobi=bs)


@pytest.mark.parametrize("bs", [4, 16])
def test_block_jacobi_cg_baseline_against_oracle(bs):
    A = W.diffusion3d(21)
    b = W.rhs(A.n, 73)
    say("pcg", A.n, bs)
    xo, io, _ = O.cg_cg(A, b, block_jacobi=bs)
    solver = M.Solver.from_matrix(A)
    x, info = solver.cg_solve(dev(b), precond=M.PRECOND_BLOCK_JACOBI, block_size=bs)
    solver.close()
    assert info["status"] == io["status"] == 0
    assert abs(info["iterations"] - io["iterations"]) <= max(1, int(np.ceil(0.01 * io["iterations"])))
    assert info["rel_res_true"] < 2e-8
    if info["iterations"] == io["iterations"]:
        assert rel(x.cpu().numpy(), xo) <= 1e-9


def test_block_jacobi_lowers_the_iteration_count():
    A = W.diffusion3d(21)
    b = W.rhs(A.n, 74)
    solver = M.Solver.from_matrix(A)
    _, i1 = solver.solve(dev(b), s=4, seed=5)
    _, i2 = solver.solve(dev(b), s=4, seed=5, precond=M.PRECOND_BLOCK_JACOBI, block_size=16)
    solver.close()
    assert i2["status"] == 0 and i2["iterations"] < i1["iterations"]


def test_block_jacobi_reports_an_indefinite_block_and_rejects_bad_sizes():
    # positive diagonal (the scaling succeeds) but the first 4 x 4 block is
    # indefinite: the setup reports NOT_SPD, as the oracle does
    A = np.eye(64)
    A[0, 1] = A[1, 0] = 2.0
    b = np.ones(64)
    _, io, _ = O.mbpcg_solve(A, b, 2, block_jacobi=4)
    assert io["status"] == O.OR_ERR_NOT_SPD
    say("indefinite block")
    solver = M.Solver.from_matrix(A)
    _, info = solver.solve(dev(b), s=2, precond=M.PRECOND_BLOCK_JACOBI, block_size=4)
    assert info["status"] == M.ERR_NOT_SPD
    _, info = solver.cg_solve(dev(b), precond=M.PRECOND_BLOCK_JACOBI, block_size=4)
    assert info["status"] == M.ERR_NOT_SPD
    for bad in (0, 2, 3, 64):
        with pytest.raises(M.MbpcgError):
            solver.solve(dev(b), s=2, precond=M.PRECOND_BLOCK_JACOBI, block_size=bad)
    with pytest.raises(M.MbpcgError):
        solver.solve(dev(b), s=2, precond=M.PRECOND_BLOCK_JACOBI, block_size=8,
                     precision=M.FP32_IR)
    solver.close()


@pytest.mark.parametrize("s", [3, 4, 8])
def test_block_iterate_against_oracle(s):
    # the block iterate X = X~ + X0 at exit (scaled space), exported on request
    A = W.diffusion3d(20)
    b = W.rhs(A.n, 75)
    seed = W.uniform_block_seed(75, s)
    runs = PC.in_variants(O.mbpcg_solve, A, b, s, seed=seed, want_X=True)
    _, io, exo = runs[0]
    say("block iterate", A.n, s)
    solver = M.Solver.from_matrix(A)
    Xg = torch.zeros((A.n, s), dtype=torch.float64, device=DEV)
    _, info = solver.solve(dev(b), s=s, seed=seed, X_out=Xg)
    Xh = np.zeros((A.n, s))
    _, info_h = solver.solve(b, s=s, seed=seed, X_out=Xh)    # host memory
    solver.close()
    assert info["iterations"] == info_h["iterations"]
    assert np.array_equal(Xg.cpu().numpy(), Xh)
    if all(info["iterations"] == r[1]["iterations"] for r in runs):
        f = PC.noise_floor(exo["X"], [r[2]["X"] for r in runs[1:]])
        err = rel(Xg.cpu().numpy(), exo["X"])
        assert err <= max(1e-10, 10 * f), (err, f)


@pytest.mark.parametrize("n,s", [(3, 8), (5, 8), (20, 32), (7, 3)])
@pytest.mark.parametrize("fmt", ["dense", "csr"])
def test_degenerate_sizes_against_oracle(n, s, fmt):
    # n <= s: the first Cholesky QR or the first iteration drops columns and
    # the residual reaches zero within a step or two
    A = W.tiny_spd(n, 50.0, tag=(80, n, s))
    b = W.rng_for((81, n)).standard_normal(n)
    M_ = A if fmt == "dense" else W.dense_to_csr(A)
    x, info, xo, io = check_against_oracle(M_, b, s, seed=3)
    assert info["rel_res_true"] < 1e-12


@pytest.mark.parametrize("s", [1, 4])
@pytest.mark.parametrize("fmt", ["dense", "csr"])
def test_one_row_system(s, fmt):
    # n = 1: X0 = gamma U can already be the solution (R0 = 0 exactly, every
    # column dropped, no iteration) or miss it by an ulp (one iteration);
    # which one depends on rounding in gamma, so only the answer is compared
    A = np.array([[2.5]])
    b = np.array([-1.75])
    say("one row", s, fmt)
    solver = M.Solver.from_matrix(A if fmt == "dense" else W.dense_to_csr(A))
    x, info = solver.solve(dev(b), s=s, seed=3)
    solver.close()
    assert info["status"] == 0 and info["iterations"] <= 1
    assert abs(x.cpu().numpy()[0] - (-0.7)) <= 1e-15


def test_explicit_block_with_duplicate_columns_deflates():
    A = W.poisson2d(16)
    b = W.rhs(A.n, 6)
    U = O.uniform_block(77, A.n, 4)
    U[:, 2] = U[:, 0]
    x, info, xo, io = check_against_oracle(A, b, 4, U=U)
    assert info["deflations"] == io["deflations"] >= 1


def test_s1_history_matches_oracle():
    A = W.poisson2d(64)
    b = W.rhs(A.n, W.CFG_POISSON2D)
    say("history s=1")
    _, io, ex = O.mbpcg_solve(A, b, 1, seed=5, want_history=True)
    solver = M.Solver.from_matrix(A)
    _, info = solver.solve(dev(b), s=1, seed=5, history=True)
    h = info["history"]
    k = min(len(h), 100)
    assert np.max(np.abs(h[:k] - ex["history"][:k]) / ex["history"][:k]) < 1e-9
    solver.close()


def test_cg_baseline_against_oracle():
    A = W.poisson2d(64)
    b = W.rhs(A.n, W.CFG_POISSON2D)
    say("cg")
    xo, io, ho = O.cg_cg(A, b, want_history=True)
    solver = M.Solver.from_matrix(A)
    x, info = solver.cg_solve(dev(b), history=True)
    x = x.cpu().numpy()
    assert info["iterations"] == io["iterations"]
    assert rel(x, xo) < 1e-9
    assert info["rel_res_true"] < 2e-8
    assert np.max(np.abs(info["history"] - ho) / ho) < 1e-8
    solver.close()


def test_cg_dense_baseline():
    A = W.dense_spd(600, tag=(3, 43))
    b = W.rng_for((3, 44)).standard_normal(600)
    say("cg dense")
    runs = PC.in_variants(O.cg_cg, A, b, jacobi=False)
    its = [r[1]["iterations"] for r in runs]
    solver = M.Solver.from_matrix(A)
    x, info = solver.cg_solve(dev(b), precond=M.PRECOND_NONE)
    # Chronopoulos-Gear CG on this spectrum moves by several steps under a
    # change of rounding; the GPU must land inside the oracle runs' range (+1)
    assert min(its) - 1 <= info["iterations"] <= max(its) + 1, (info["iterations"], its)
    assert info["rel_res_true"] < 2e-8
    solver.close()


# -------------------------------------------------------------- edge cases
def test_zero_rhs():
    A = W.poisson2d(8)
    say("zero rhs")
    solver = M.Solver.from_matrix(A)
    x, info = solver.solve(torch.zeros(A.n, dtype=torch.float64, device=DEV), s=4)
    assert info["status"] == 0 and info["iterations"] == 0 and not x.any().item()
    solver.close()


def test_nonfinite_rhs():
    A = W.poisson2d(8)
    b = np.ones(A.n)
    b[3] = np.nan
    say("nan rhs")
    solver = M.Solver.from_matrix(A)
    _, info = solver.solve(dev(b), s=2)
    assert info["status"] == M.ERR_NONFINITE
    solver.close()


def test_nonpositive_diagonal():
    A = W.poisson2d(8)
    A.vals = A.vals.copy()
    A.vals[A.colind == 0] = -1.0
    say("not spd")
    solver = M.Solver.from_matrix(A)
    _, info = solver.solve(dev(np.ones(A.n)), s=2)
    assert info["status"] == M.ERR_NOT_SPD
    solver.close()


@pytest.mark.parametrize("kind", ["tridiagonal", "shifted_poisson"])
@pytest.mark.parametrize("s", [1, 2, 4])
def test_indefinite_matrix_stops_not_spd_with_the_best_column(kind, s):
    # positive diagonals, indefinite matrices: tridiagonal (1, -0.9) with 156
    # of 500 eigenvalues negative, where P^T A P fails at the first step; the
    # 16 x 16 Poisson matrix minus 0.1 I with one negative eigenvalue, where
    # it fails after a dozen steps.  The failing step's update never runs;
    # the best column of the iterate so far is returned.
    import scipy.sparse as sp
    if kind == "tridiagonal":
        n = 500
        T = sp.diags([-0.9 * np.ones(n - 1), np.ones(n), -0.9 * np.ones(n - 1)], [-1, 0, 1])
    else:
        P = W.poisson2d(16)
        n = P.n
        T = sp.csr_matrix((P.vals, P.colind, P.rowptr), shape=(n, n)) - 0.1 * sp.identity(n)
    T = T.tocsr()
    T.sort_indices()
    A = W.CSR(n, T.indptr.astype(np.int32), T.indices.astype(np.int32), T.data.astype(np.float64))
    b = W.rhs(n, 5)
    x, info, xo, io = check_against_oracle(A, b, s, seed=3)
    assert io["status"] == M.ERR_NOT_SPD and info["status"] == M.ERR_NOT_SPD
    assert info["used_fallback"] == 1 and info["iterations"] == io["iterations"]


def test_max_iter_returns_best_column():
    A = W.diffusion3d(12)
    b = W.rhs(A.n, 5)
    say("max_iter")
    x, info, xo, io = check_against_oracle(A, b, 4, seed=1, max_iter=7)
    assert info["status"] == 1 and info["iterations"] == 7 and info["used_fallback"] == 1


def test_host_memory_path():
    A = W.poisson2d(32)
    b = W.rhs(A.n, 8)
    say("host memory")
    xo, io, _ = O.mbpcg_solve(A, b, 4, seed=2)
    solver = M.Solver.from_matrix(A)
    x, info = solver.solve(b, s=4, seed=2)
    assert isinstance(x, np.ndarray)
    assert info["iterations"] == io["iterations"] and rel(x, xo) < 1e-10
    solver.close()


def test_repeat_solves_are_bitwise_identical():
    A = W.diffusion3d(16)
    b = W.rhs(A.n, 9)
    say("determinism")
    solver = M.Solver.from_matrix(A)
    x1, i1 = solver.solve(dev(b), s=8, seed=3)
    x2, i2 = solver.solve(dev(b), s=8, seed=3)
    assert i1["iterations"] == i2["iterations"]
    assert torch.equal(x1, x2)
    solver.close()


def test_launch_modes_give_the_same_solve():
    # graph mode, every phase timed, and only the block product timed: the
    # same kernels in the same order, so bitwise the same x
    A = W.diffusion3d(16)
    b = W.rhs(A.n, 9)
    say("launch modes")
    solver = M.Solver.from_matrix(A)
    x0, i0 = solver.solve(dev(b), s=4, seed=3)
    x1, i1 = solver.solve(dev(b), s=4, seed=3, profile=1)
    x2, i2 = solver.solve(dev(b), s=4, seed=3, profile=2)
    assert i0["iterations"] == i1["iterations"] == i2["iterations"]
    assert torch.equal(x0, x1) and torch.equal(x0, x2)
    assert i2["spmm_launches"] == i1["spmm_launches"] > 0 and i2["ms_spmm"] > 0
    assert all(v > 0 for v in i1["ms_phase"][:5])
    assert all(v == 0 for v in i2["ms_phase"][1:5]) and i2["ms_phase"][0] > 0
    c1, j1 = solver.cg_solve(dev(b), profile=1)
    c2, j2 = solver.cg_solve(dev(b), profile=2)
    assert j1["iterations"] == j2["iterations"] and torch.equal(c1, c2)
    assert j2["spmm_launches"] == j1["spmm_launches"] > 0 and j2["ms_spmm"] > 0
    solver.close()


# ------------------------------------------------------ mixed precision (IR)
def test_fp32_iterative_refinement_reaches_1e10():
    n = 512
    A = W.dense_spd(n, tag=(4, 50))
    b = W.rng_for((4, 51)).standard_normal(n)
    say("fp32 IR", n)
    xs = np.linalg.solve(A, b)
    solver = M.Solver.from_matrix(A)
    x, info = solver.solve(dev(b), s=8, precision=M.FP32_IR, precond=M.PRECOND_NONE,
                           ir_tol=1e-10, inner_tol=1e-5, seed=4)
    x = x.cpu().numpy()
    assert info["status"] == 0, info
    assert info["rel_res_true"] <= 1e-10
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) <= 2e-10
    assert rel(x, xs) <= np.linalg.cond(A) * 1e-10
    solver.close()


def test_fp32_iterative_refinement_against_the_oracle():
    # the oracle's refinement loop with FP32-rounded products (same inner
    # tolerance rule, same inner seeds): equal outer steps, total inner
    # iterations within 5 %, and both at the FP64 tolerance, so the two x
    # differ by at most 2 kappa ir_tol
    n = 1024
    A = W.dense_spd(n, tag=(4, 60))
    b = W.rng_for((4, 61)).standard_normal(n)
    say("fp32 IR vs oracle", n)
    xo, io = O.ir_solve(A, b, 8, O.LO_FP32, ir_tol=1e-10, seed=6)
    solver = M.Solver.from_matrix(A)
    x, info = solver.solve(dev(b), s=8, precision=M.FP32_IR, precond=M.PRECOND_NONE,
                           ir_tol=1e-10, seed=6)
    x = x.cpu().numpy()
    assert info["status"] == io["status"] == 0, (info, io)
    assert info["outer_iterations"] == io["outer_iterations"], (info, io)
    assert abs(info["iterations"] - io["iterations"]) <= np.ceil(0.05 * io["iterations"]), (info, io)
    kappa = np.linalg.cond(A)
    assert rel(x, xo) <= 2 * kappa * 1e-10
    solver.close()


def test_bf16_iterative_refinement_against_the_oracle():
    A = W.tiny_spd(613, 20.0, tag=(4, 62))
    b = W.rng_for((4, 63)).standard_normal(613)
    say("bf16 IR vs oracle", 613)
    xo, io = O.ir_solve(A, b, 8, O.LO_BF16, ir_tol=1e-10, seed=7)
    solver = M.Solver.from_matrix(A)
    x, info = solver.solve(dev(b), s=8, precision=M.BF16_IR, precond=M.PRECOND_NONE,
                           ir_tol=1e-10, seed=7)
    x = x.cpu().numpy()
    assert info["status"] == io["status"] == 0, (info, io)
    assert abs(info["outer_iterations"] - io["outer_iterations"]) <= 1, (info, io)
    assert abs(info["iterations"] - io["iterations"]) <= np.ceil(0.10 * io["iterations"]), (info, io)
    assert rel(x, xo) <= 2 * np.linalg.cond(A) * 1e-10
    solver.close()


@pytest.mark.parametrize("prec,n", [("fp32", 613), ("bf16", 600)])
def test_low_precision_refinement_odd_k_steps_against_the_oracle(prec, n):
    # orders whose column ranges hold an odd number of k-steps (FP32: 39
    # steps of 16 over two ranges, 20 + 19; BF16: 19 steps of 32, 10 + 9)
    # and a ragged last row tile: the products' final single step and the
    # clamped operand rows, against the oracle's refinement with products
    # rounded the same way
    A = W.tiny_spd(n, 20.0, tag=(4, 64, n))
    b = W.rng_for((4, 65, n)).standard_normal(n)
    say("low-precision IR vs oracle, odd k-steps", prec, n)
    lo = O.LO_FP32 if prec == "fp32" else O.LO_BF16
    xo, io = O.ir_solve(A, b, 8, lo, ir_tol=1e-10, seed=8)
    solver = M.Solver.from_matrix(A)
    x, info = solver.solve(dev(b), s=8, precision=M.FP32_IR if prec == "fp32" else M.BF16_IR,
                           precond=M.PRECOND_NONE, ir_tol=1e-10, seed=8)
    x = x.cpu().numpy()
    assert info["status"] == io["status"] == 0, (info, io)
    assert abs(info["outer_iterations"] - io["outer_iterations"]) <= (0 if prec == "fp32" else 1)
    band = 0.05 if prec == "fp32" else 0.10
    assert abs(info["iterations"] - io["iterations"]) <= np.ceil(band * io["iterations"]), (info, io)
    assert rel(x, xo) <= 2 * np.linalg.cond(A) * 1e-10
    solver.close()


def test_bf16_iterative_refinement_reports_honestly():
    n = 256
    A = W.dense_spd(n, tag=(4, 52))
    b = W.rng_for((4, 53)).standard_normal(n)
    say("bf16 IR", n)
    solver = M.Solver.from_matrix(A)
    x, info = solver.solve(dev(b), s=8, precision=M.BF16_IR, precond=M.PRECOND_NONE,
                           ir_tol=1e-10, inner_tol=1e-2, max_outer=30, seed=4)
    x = x.cpu().numpy()
    truth = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    # whatever the outcome, the reported FP64 residual is the true one, and an
    # outer step that does not lower it is taken back (never worse than x = 0)
    assert abs(truth - info["rel_res_true"]) <= 1e-6 * max(truth, 1e-12) + 1e-14
    assert truth <= 1.0
    if info["status"] == 0:
        assert truth <= 2e-10
    solver.close()


@pytest.mark.parametrize("prec,n,s", [("fp32", 300, 4), ("fp32", 613, 32), ("bf16", 300, 16),
                                      ("bf16", 613, 8)])
def test_low_precision_products_on_ragged_orders(prec, n, s):
    # orders that are not multiples of the 16/32-wide tiles of the
    # low-precision copies, one and two 16-column MFMA tiles; a system
    # conditioned so that even BF16 products make the refinement contract
    A = W.tiny_spd(n, 20.0, tag=(4, 54, n))
    b = W.rng_for((4, 55, n)).standard_normal(n)
    say("low-precision IR", prec, n, s)
    solver = M.Solver.from_matrix(A)
    x, info = solver.solve(dev(b), s=s, precision=M.FP32_IR if prec == "fp32" else M.BF16_IR,
                           precond=M.PRECOND_NONE, ir_tol=1e-10, seed=5)
    x = x.cpu().numpy()
    truth = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert info["status"] == 0, info
    assert truth <= 2e-10
    assert abs(truth - info["rel_res_true"]) <= 1e-6 * truth + 1e-14
    solver.close()
