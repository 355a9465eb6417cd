"""Full-size parity: the configured workloads solved on the GPU, in the launch
configuration the benchmark times, against the oracle's stored results for
the same seeded input bytes.

The golden files are written by tests/golden/make_*_golden.py from the CPU
oracle alone.  Each solve there runs in the oracle's three rounding
variants (reference, blocked-pairwise sums, fused multiply-adds); a record
holds their iteration counts, the noise floor (largest relative distance
between two variants' x) and x at fixed sampled indices.  The bar is the
parity contract of the small tests (parity_contract.check_golden):
iteration counts within the variants' range (+1 when the deciding residual
is within 1 % of tol), and where the count equals a variant's, the sampled
x within max(1e-10, 10 x noise floor) of that variant's.

* 128^3 diffusion (n = 2.1M), s = 1, 2, 4, 8, 16 and CG, profile and graph mode
* dense n = 8192, s = 1, 4, 8, 16, 32 and CG (the column-range split of the
  full-size dense product)
* dense n = 16384 mixed precision: FP32 iterative refinement to 1e-10 at
  s = 8, 16, 32 against the oracle's FP64 reference solution (tol 1e-12,
  cross-checked with LAPACK) and its FP32-emulating refinement
* the 512-system batch in one persistent launch, every system
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import parity_contract as PC
from paper_2608_07327_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2608_07327_amd import mbpcg as M  # noqa: E402

DEV = torch.device("cuda:0")
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def load(name):
    return json.load(open(os.path.join(GOLD, name)))


def sha(*arrays):
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


# ------------------------------------------------------------ 128^3 diffusion
@pytest.fixture(scope="module")
def diffusion():
    gold = load("diffusion3d_128.json")
    A = W.diffusion3d(gold["grid"])
    b = W.rhs(A.n, W.CFG_DIFFUSION3D)
    # the stored results belong to exactly these input bytes
    assert sha(A.rowptr, A.colind, A.vals, b) == gold["input_sha256"]
    solver = M.Solver.from_matrix(A)
    bd = torch.as_tensor(b, device=DEV)
    yield gold, solver, bd, np.asarray(gold["sample_index"])
    solver.close()


@pytest.mark.parametrize("s", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("mode", ["profile", "graph"])
def test_full_size_diffusion_against_oracle_golden(diffusion, s, mode):
    gold, solver, bd, idx = diffusion
    o = gold["mbpcg"][str(s)]
    say("golden 128^3", s, mode)
    solver.autotune(s)
    x, info = solver.solve(bd, s=s, seed=o["seed"], profile=1 if mode == "profile" else 0)
    PC.check_golden(x.cpu().numpy()[idx], info, o, 1e-8, what=f"128^3 s={s} {mode}")


def test_full_size_diffusion_cg_against_oracle_golden(diffusion):
    gold, solver, bd, idx = diffusion
    say("golden 128^3 CG")
    x, info = solver.cg_solve(bd, profile=1)
    PC.check_golden(x.cpu().numpy()[idx], info, gold["cg"], 1e-8, what="128^3 CG")


# --------------------------------------------------------------- dense 8192
@pytest.fixture(scope="module")
def dense8192():
    gold = load("dense_8192.json")
    n = gold["n"]
    say("dense 8192 inputs")
    A = W.dense_spd_torch(n, W.CFG_DENSE, gold["shift"], device=DEV)
    b = W.rhs(n, W.CFG_DENSE)
    assert sha(A.cpu().numpy(), b) == gold["input_sha256"]
    solver = M.Solver.from_dense(A)
    bd = torch.as_tensor(b, device=DEV)
    yield gold, solver, bd, np.asarray(gold["sample_index"])
    solver.close()
    del A
    torch.cuda.empty_cache()


@pytest.mark.parametrize("s", [1, 4, 8, 16, 32])
def test_full_size_dense_against_oracle_golden(dense8192, s):
    gold, solver, bd, idx = dense8192
    o = gold["mbpcg"][str(s)]
    say("golden dense 8192", s)
    x, info = solver.solve(bd, s=s, tol=gold["tol"], precond=M.PRECOND_NONE, seed=o["seed"],
                           profile=1)
    PC.check_golden(x.cpu().numpy()[idx], info, o, gold["tol"], what=f"dense s={s}")


def test_full_size_dense_cg_against_oracle_golden(dense8192):
    gold, solver, bd, idx = dense8192
    say("golden dense 8192 CG")
    x, info = solver.cg_solve(bd, tol=gold["tol"], precond=M.PRECOND_NONE, profile=1)
    PC.check_golden(x.cpu().numpy()[idx], info, gold["cg"], gold["tol"], what="dense CG")


# ------------------------------------------------------ dense 16384, mixed
@pytest.fixture(scope="module")
def dense16384():
    gold = load("dense_mixed_16384.json")
    n = gold["n"]
    say("dense 16384 inputs")
    A = W.dense_spd_torch(n, W.CFG_DENSE_MIXED, gold["shift"], device=DEV)
    b = W.rhs(n, W.CFG_DENSE_MIXED)
    assert sha(A.cpu().numpy(), b) == gold["input_sha256"]
    solver = M.Solver.from_dense(A)
    bd = torch.as_tensor(b, device=DEV)
    yield gold, solver, bd, np.asarray(gold["sample_index"])
    solver.close()
    del A
    torch.cuda.empty_cache()


def test_fp64_oracle_reference_is_the_direct_solution(dense16384):
    # the stored reference (oracle MBPCG to 1e-12) against LAPACK's solve,
    # both computed when the golden file was written
    gold = dense16384[0]
    assert gold["ref"]["status"] == 0 and gold["ref"]["rel_res_true"] < 2 * gold["ref_tol"]
    assert gold["ref"]["vs_numpy_solve"] < 4e3 * 1e-12 * 10


@pytest.mark.parametrize("s", [8, 16, 32])
def test_full_size_fp32_refinement_against_fp64_oracle(dense16384, s):
    gold, solver, bd, idx = dense16384
    if str(s) not in gold["ir_fp32"] or str(s) not in gold.get("ir_fp32_pairwise", {}):
        pytest.skip("the oracle's FP32-emulating refinement is not recorded for this width")
    o = gold["ir_fp32"][str(s)]
    say("golden dense 16384 FP32 IR", s)
    x, info = solver.solve(bd, s=s, precision=M.FP32_IR, ir_tol=gold["ir_tol"],
                           inner_tol=gold["inner_tol"], precond=M.PRECOND_NONE, seed=o["seed"],
                           profile=1)
    assert info["status"] == 0 and info["rel_res_true"] <= gold["ir_tol"]
    # error against the FP64 oracle solution: the refinement stops at
    # ||b - A x|| <= 1e-10 ||b||, so ||x - x*|| <= kappa 1e-10 ||x*||, kappa
    # ~ 4e3 (Marchenko-Pastur edge 4 over the shift 1e-3)
    xs = x.cpu().numpy()[idx]
    xr = np.asarray(gold["ref"]["x_sample"])
    err = float(np.linalg.norm(xs - xr) / np.linalg.norm(xr))
    say("  error vs FP64 oracle", err, "oracle's FP32 emulation", o["err_vs_ref"])
    assert err <= 4e3 * gold["ir_tol"]
    # inner iterations within 5 % of the range spanned by the oracle's
    # FP32-emulating refinements (A and the blocks rounded to FP32 as on the
    # GPU; FP32 sums over the 16384 columns sequential or blocked-pairwise --
    # the order alone moves the inner count by ~10 %, the GPU sums in blocks)
    its = [o["iterations"]]
    op = gold.get("ir_fp32_pairwise", {}).get(str(s))
    if op is not None:
        its.append(op["iterations"])
    lo, hi = 0.95 * min(its), 1.05 * max(its)
    assert lo <= info["iterations"] <= hi, (info["iterations"], its)
    assert min(o["outer_iterations"], (op or o)["outer_iterations"]) - 1 <= \
        info["outer_iterations"] <= max(o["outer_iterations"], (op or o)["outer_iterations"]) + 1


def test_full_size_fp64_cg_against_fp64_oracle(dense16384):
    gold, solver, bd, idx = dense16384
    say("golden dense 16384 FP64 CG to 1e-10")
    x, info = solver.cg_solve(bd, tol=gold["ir_tol"], precond=M.PRECOND_NONE)
    assert info["status"] == 0
    xs = x.cpu().numpy()[idx]
    xr = np.asarray(gold["ref"]["x_sample"])
    assert np.linalg.norm(xs - xr) / np.linalg.norm(xr) <= 4e3 * gold["ir_tol"]


# ---------------------------------------------------------------- batch 512
def test_full_size_batch_against_oracle_golden():
    gold = load("batch_512.json")
    say("golden batch: generating", gold["count"], "systems")
    systems = W.graph_laplacian_batch(count=gold["count"])
    h = hashlib.sha256()
    for y in systems:
        for a in (y.A.rowptr, y.A.colind, y.A.vals, y.b):
            h.update(np.ascontiguousarray(a).tobytes())
        h.update(np.int64(y.s).tobytes())
    assert h.hexdigest() == gold["input_sha256"]
    items = []
    for y in systems:
        items.append(dict(n=y.A.n, rowptr=torch.as_tensor(y.A.rowptr, device=DEV),
                          colind=torch.as_tensor(y.A.colind, device=DEV),
                          vals=torch.as_tensor(y.A.vals, device=DEV),
                          b=torch.as_tensor(y.b, device=DEV),
                          x=torch.zeros(y.A.n, dtype=torch.float64, device=DEV), s=y.s))
    say("golden batch: one persistent launch")
    st, infos = M.solve_batch(items, seed=gold["seed"])
    assert st == 0
    compared = 0
    for i, (it, info, o) in enumerate(zip(items, infos, gold["systems"])):
        err = PC.check_golden(it["x"].cpu().numpy()[np.asarray(o["sample_index"])], info, o,
                              1e-8, what=f"batch system {i}")
        compared += err is not None
    say("golden batch: x compared on", compared, "of", len(items), "systems")
    assert compared >= 0.9 * len(items)
