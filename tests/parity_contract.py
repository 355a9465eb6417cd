"""The FP64 parity contract between a GPU solve and the CPU oracle.

The oracle runs twice on the same input, with sequential and with
blocked-pairwise reductions; that pair fixes how much the method itself
moves when only the rounding order changes (its noise floor).  The GPU adds
in yet another fixed order and is held to that band:

* status equal;
* iteration count within |it_seq - it_pairwise|, plus 1 when the best
  column's relative residual at the deciding iteration (the last one, or the
  one before it) is within 1 % of tol;
* when the GPU's count equals the oracle's (either ordering's): x within
  max(floor, 10 f) of that ordering's x, with f = |x_pairwise - x_seq| /
  |x_seq| and floor 1e-10; used_fallback,
  final_width and deflations equal wherever the two oracle orderings agree
  on them;
* converged solves: FP64 true residual below 2 tol.

No case is exempt: the least squares of the termination computes the same
minimiser on both sides (the GPU's Gram is double-double, so the columns'
independent parts are resolved as the oracle's Householder QR resolves
them), and the fallback to the best column on the true residual is the same
rule on both sides.
"""
import numpy as np

from oracle import oracle as O


def oracle_band(A, b, s, **kw):
    """Oracle run with sequential and with blocked-pairwise reductions;
    returns (x_seq, info_seq, x_pair, info_pair) with the best-column
    residual histories in info['history']."""
    xs, i_s, es = O.mbpcg_solve(A, b, s, want_history=True, **kw)
    O.set_summation(1)
    try:
        xp, i_p, ep = O.mbpcg_solve(A, b, s, want_history=True, **kw)
    finally:
        O.set_summation(0)
    i_s["history"] = es["history"]
    i_p["history"] = ep["history"]
    return xs, i_s, xp, i_p


def near_tol(io, tol):
    """The best column's residual at the deciding iteration, or the one
    before it, within 1 % of tol (another rounding order may stop one
    iteration later or earlier)."""
    h = np.asarray(io.get("history", []))
    vals = [io["rel_res_best"]] + ([h[-2]] if h.size >= 2 else [])
    return any(abs(v - tol) <= 0.01 * tol for v in vals)


def iteration_band(io, ip, tol):
    return abs(io["iterations"] - ip["iterations"]) + (1 if near_tol(io, tol) else 0)


def rel(a, b):
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def check(x, info, xo, io, xp, ip, tol, floor=1e-10, what=""):
    """Assert the contract above; returns the measured |x - x_seq| / |x_seq|
    (None when the counts differ)."""
    assert info["status"] == io["status"], (what, info, io)
    band = iteration_band(io, ip, tol)
    assert abs(info["iterations"] - io["iterations"]) <= band, \
        (what, info["iterations"], io["iterations"], ip["iterations"])
    err = None
    f = rel(xp, xo)
    for ref, iref in ((xo, io), (xp, ip)):
        # against the oracle ordering that took the same number of steps
        if info["iterations"] == iref["iterations"]:
            err = rel(x, ref)
            assert err <= max(floor, 10 * f), (what, err, f)
            for key in ("used_fallback", "final_width", "deflations"):
                if io[key] == ip[key]:
                    assert info[key] == iref[key], (what, key, info[key], iref[key])
            break
    if io["status"] == 0:
        assert info["rel_res_true"] < 2 * tol, (what, info["rel_res_true"])
    return err
