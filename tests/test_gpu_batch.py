"""Batched solve (one persistent kernel) vs the oracle run system by system.

System i of a batch draws its initial block from SplitMix64 seeded with
common_seed + i.  Each system is held to the same contract as a single
solve (parity_contract.check): iteration count inside the oracle's own
rounding-order band, solution within max(1e-10, 10 f) when the counts
agree, true residual below 2 tol.
"""
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


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV)


def to_items(systems):
    items = []
    for y in systems:
        items.append(dict(n=y.A.n, rowptr=dev(y.A.rowptr), colind=dev(y.A.colind),
                          vals=dev(y.A.vals), b=dev(y.b),
                          x=torch.zeros(y.A.n, dtype=torch.float64, device=DEV), s=y.s))
    return items


def check_batch(systems, seed=100, floor=1e-10):
    """Every system of one batched solve against the oracle's two orderings
    for that system (parity_contract.check)."""
    items = to_items(systems)
    say("batch", len(items), [(y.A.n, y.s) for y in systems])
    st, infos = M.solve_batch(items, seed=seed)
    for i, (y, it, info) in enumerate(zip(systems, items, infos)):
        xo, io, xp, ip = PC.oracle_band(y.A, y.b, y.s, seed=seed + i)
        x = it["x"].cpu().numpy()
        if not np.any(xo):
            assert info["status"] == io["status"] and not np.any(x), i
            continue
        PC.check(x, info, xo, io, xp, ip, 1e-8, floor=floor, what=f"system {i}")
    return st, infos


def test_batch_of_graph_laplacians():
    systems = W.graph_laplacian_batch(count=12, n_lo=200, n_hi=5000, tag=(5, 1))
    st, infos = check_batch(systems)
    assert st == 0


def test_batch_padded_widths_against_oracle():
    # s = 5, 6, 7 carried at the padded width 8, s = 2 at 2, beside each
    # other in one launch
    A = W.poisson2d(40)
    B3 = W.diffusion3d(14)
    sys_list = [W.BatchSystem(A, W.rhs(A.n, 51), 5), W.BatchSystem(B3, W.rhs(B3.n, 52), 6),
                W.BatchSystem(A, W.rhs(A.n, 53), 7), W.BatchSystem(B3, W.rhs(B3.n, 54), 2)]
    st, infos = check_batch(sys_list, seed=300)
    assert st == 0


def test_batch_mixes_stencils_widths_and_edge_cases():
    A = W.poisson2d(32)
    sys_list = [
        W.BatchSystem(A, W.rhs(A.n, 31), 4),
        W.BatchSystem(A, W.rhs(A.n, 32), 1),
        W.BatchSystem(A, np.zeros(A.n), 8),                        # b = 0
        W.BatchSystem(W.diffusion3d(11), W.rhs(11 ** 3, 33), 2),
        W.BatchSystem(W.diffusion3d(7), W.rhs(7 ** 3, 34), 3),     # padded width
    ]
    st, infos = check_batch(sys_list, seed=7)
    assert infos[2]["iterations"] == 0 and infos[2]["status"] == 0


def test_batch_near_singular_laplacians_against_oracle():
    # Laplacians shifted by 1e-6 (kappa ~ 1.6e7): the termination's least
    # squares on nearly dependent columns and the true-residual fallback,
    # every system against its oracle solve
    sys_list = []
    for k, (n, s) in enumerate([(2000, 2), (2000, 8), (5000, 4), (1200, 1)]):
        A = W.graph_laplacian(n, 8, 1e-6, W.rng_for((W.CFG_BATCH, 98, n, k)))
        sys_list.append(W.BatchSystem(A, W.rng_for((99, k)).standard_normal(n), s))
    st, infos = check_batch(sys_list, seed=21)
    assert st == 0


def test_batch_context_replays_and_matches_the_one_call_solve():
    # a batch context uploads once and replays its graph: repeated solves
    # are bitwise the one-call solve's
    systems = W.graph_laplacian_batch(count=6, n_lo=300, n_hi=4000, tag=(5, 3))
    items = to_items(systems)
    say("batch context")
    st0, i0 = M.solve_batch(items, seed=31)
    x0 = [it["x"].clone() for it in items]
    with M.Batch(items) as bt:
        for rep in range(3):
            for it in items:
                it["x"].zero_()
            st, infos = bt.solve(seed=31, profile=rep == 1)
            assert st == st0
            for a, b2, ia, ib in zip(items, x0, infos, i0):
                assert ia["iterations"] == ib["iterations"]
                assert torch.equal(a["x"], b2)


def test_batch_autotune_then_parity():
    # the tuned lane groups per row and grid change only the summation order:
    # every system still meets the parity contract
    systems = W.graph_laplacian_batch(count=8, n_lo=300, n_hi=6000, tag=(5, 4))
    # one system with long rows (dense block) so two row classes are present
    A = W.dense_to_csr(W.dense_spd(40, tag=(5, 41)))
    systems.append(W.BatchSystem(A, W.rng_for((5, 42)).standard_normal(40), 4))
    items = to_items(systems)
    say("batch autotune")
    with M.Batch(items) as bt:
        t = bt.autotune(seed=40)
        assert t["trials"] >= 1 and t["workgroups"] >= 1 and t["classes"] >= 2
        st, infos = bt.solve(seed=40)
    for i, (y, it, info) in enumerate(zip(systems, items, infos)):
        xo, io, xp, ip = PC.oracle_band(y.A, y.b, y.s, seed=40 + i)
        PC.check(it["x"].cpu().numpy(), info, xo, io, xp, ip, 1e-8, what=f"tuned system {i}")


def test_batch_matches_single_solves():
    systems = W.graph_laplacian_batch(count=4, n_lo=500, n_hi=3000, tag=(5, 2))
    items = to_items(systems)
    say("batch vs single")
    _, infos = M.solve_batch(items, seed=11)
    for i, (y, it, info) in enumerate(zip(systems, items, infos)):
        solver = M.Solver.from_matrix(y.A)
        x1, i1 = solver.solve(dev(y.b), s=y.s, seed=11 + i)
        solver.close()
        assert abs(i1["iterations"] - info["iterations"]) <= 1
        if i1["iterations"] == info["iterations"]:
            xb = it["x"].cpu().numpy()
            assert np.linalg.norm(xb - x1.cpu().numpy()) <= 1e-9 * np.linalg.norm(xb)


def test_width_selector_measures_on_the_gpu():
    # the measurement half of the width model runs end to end and records
    # converged CG and MBPCG solves (fitting is covered on the CPU)
    from paper_2608_07327_amd import selector as SEL
    say("width selector")
    recs = SEL.measure([("poisson2d m=24", lambda: W.poisson2d(24)),
                        ("dense n=200", lambda: W.dense_spd(200, tag=(6, 1)))],
                       widths=(2, 4), reps=1)
    assert len(recs) == 2
    for r in recs:
        assert r["cg_status"] == 0 and r["cg_iterations"] > 0 and r["cg_seconds"] > 0
        for s in ("2", "4"):
            m = r["mbpcg"][s]
            assert m["status"] == 0 and m["rel_res_true"] < 2e-8 and m["seconds"] > 0


def test_barrier_bound_ends_the_launch_and_the_next_solve_recovers(monkeypatch):
    # a wait beyond the grid barrier's bound (lowered from the host to one
    # poll) makes every workgroup exit and the call report it; the context's
    # next solve starts afresh and is bitwise the one-call solve
    systems = W.graph_laplacian_batch(count=6, n_lo=300, n_hi=4000, tag=(5, 6))
    items = to_items(systems)
    say("batch barrier bound")
    st0, i0 = M.solve_batch(items, seed=51)
    x0 = [it["x"].clone() for it in items]
    with M.Batch(items) as bt:
        monkeypatch.setenv("MBPCG_BATCH_SPIN_LIMIT", "1")
        with pytest.raises(M.MbpcgError) as err:
            bt.solve(seed=51)
        assert "grid barrier" in str(err.value)
        monkeypatch.delenv("MBPCG_BATCH_SPIN_LIMIT")
        for it in items:
            it["x"].zero_()
        st, infos = bt.solve(seed=51)
        assert st == st0
        for a, b2, ia, ib in zip(items, x0, infos, i0):
            assert ia["iterations"] == ib["iterations"]
            assert torch.equal(a["x"], b2)
