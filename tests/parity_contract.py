"""The FP64 parity contract between a GPU solve and the CPU oracle.

The oracle runs three times on the same input, in three roundings of the
same arithmetic: sequential sums with every product and sum rounded (the
reference), blocked-pairwise sums over the n rows and the dense product's
n columns, and sequential sums with multiply-adds fused.  Their spread fixes
how much the method itself moves when only the rounding changes (its noise
floor).  The GPU, which sums in fixed trees and fuses multiply-adds, is held
to that band:

* status equal;
* iteration count within the three runs' range (max - min), plus 1 when the
  best column's relative residual at the deciding iteration (the last one,
  or the one before it) is within 1 % of tol, around the reference count;
* when the GPU's count equals one of the runs' counts: x within
  max(floor, 10 f) of that run's x, with f the largest relative distance
  between two of the three runs' x and floor 1e-10 -- both normwise and
  entry by entry (the largest entry difference over the largest entry,
  against the same measure between the runs); used_fallback, final_width
  and deflations equal wherever the three runs agree on them;
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
    """The oracle in its three rounding variants; returns (x_seq, info_seq,
    x_others, info_others) with the best-column residual histories in
    info['history'] (the others: pairwise, fused multiply-add)."""
    runs = []
    try:
        for v in O.VARIANTS:
            O.set_variant(v)
            x, i, e = O.mbpcg_solve(A, b, s, want_history=True, **kw)
            i["history"] = e["history"]
            i["variant"] = v
            runs.append((x, i))
    finally:
        O.set_variant("seq")
    (xs, i_s), others = runs[0], runs[1:]
    return xs, i_s, [x for x, _ in others], [i for _, i in others]


def in_variants(fn, *a, **kw):
    """fn(*a, **kw) under each rounding variant of the oracle, reference first."""
    out = []
    try:
        for v in O.VARIANTS:
            O.set_variant(v)
            out.append(fn(*a, **kw))
    finally:
        O.set_variant("seq")
    return out


def near_tol(io, tol):
    """The best column's residual at the deciding iteration, or the one
    before it, within 1 % of tol (another rounding order may stop one
    iteration later or earlier)."""
    h = np.asarray(io.get("history", []))
    vals = [io["rel_res_best"]] + ([h[-2]] if h.size >= 2 else [])
    return any(abs(v - tol) <= 0.01 * tol for v in vals)


def iteration_band(io, ips, tol):
    its = [io["iterations"]] + [ip["iterations"] for ip in ips]
    return max(its) - min(its) + (1 if near_tol(io, tol) else 0)


def rel(a, b):
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def noise_floor(xo, xps):
    xs = [xo] + list(xps)
    nb = float(np.linalg.norm(xo))
    if nb == 0.0:
        return 0.0
    return max(float(np.linalg.norm(a - c)) / nb for k, a in enumerate(xs) for c in xs[k + 1:])


def noise_floor_entries(xo, xps):
    """The noise floor entry by entry: the largest difference of one entry
    between two runs, over the reference run's largest entry."""
    xs = [np.asarray(xo)] + [np.asarray(v) for v in xps]
    m = float(np.max(np.abs(xs[0]))) if xs[0].size else 0.0
    if m == 0.0:
        return 0.0
    return max(float(np.max(np.abs(a - c))) / m for k, a in enumerate(xs) for c in xs[k + 1:])


def rel_entries(a, b):
    m = float(np.max(np.abs(b))) if np.asarray(b).size else 0.0
    d = float(np.max(np.abs(np.asarray(a) - np.asarray(b)))) if np.asarray(b).size else 0.0
    return d / m if m > 0 else d


def check(x, info, xo, io, xps, ips, tol, floor=1e-10, what=""):
    """Assert the contract above; returns the measured |x - x_ref| / |x_ref|
    against the run with the same count (None when no run has it)."""
    assert info["status"] == io["status"], (what, info, io)
    band = iteration_band(io, ips, tol)
    assert abs(info["iterations"] - io["iterations"]) <= band, \
        (what, info["iterations"], io["iterations"], [ip["iterations"] for ip in ips])
    f = noise_floor(xo, xps)
    err = None
    for ref, iref in [(xo, io)] + list(zip(xps, ips)):
        # against an oracle run that took the same number of steps
        if info["iterations"] == iref["iterations"]:
            err = rel(x, ref)
            assert err <= max(floor, 10 * f), (what, iref.get("variant"), err, f)
            fe = noise_floor_entries(xo, xps)
            ee = rel_entries(x, ref)
            assert ee <= max(floor, 10 * fe), (what, "entries", iref.get("variant"), ee, fe)
            for key in ("used_fallback", "final_width", "deflations"):
                if all(ip[key] == io[key] for ip in ips):
                    assert info[key] == iref[key], (what, key, info[key], iref[key])
            break
    if io["status"] == 0:
        assert info["rel_res_true"] < 2 * tol, (what, info["rel_res_true"])
    return err


def check_golden(x_sample, info, o, tol, floor=1e-10, what=""):
    """The same contract against a stored oracle record (golden file written
    by tests/golden/*: the reference run's diagnostics, the three variants'
    counts and sampled x, the noise floor over the full vectors).  x_sample
    is the GPU's x at the record's sample indices."""
    assert info["status"] == o["status"], (what, info["status"], o["status"])
    its = [o["iterations"], o["pairwise_iterations"], o["fma_iterations"]]
    near = abs(o["rel_res_best"] - tol) <= 0.01 * tol
    band = max(its) - min(its) + (1 if near else 0)
    assert abs(info["iterations"] - o["iterations"]) <= band, (what, info["iterations"], its)
    err = None
    for key, xsk in (("iterations", "x_sample"), ("pairwise_iterations", "pairwise_x_sample"),
                     ("fma_iterations", "fma_x_sample")):
        if info["iterations"] == o[key]:
            xr = np.asarray(o[xsk])
            err = float(np.linalg.norm(np.asarray(x_sample) - xr) / np.linalg.norm(xr))
            assert err <= max(floor, 10 * o["noise_floor"]), (what, key, err, o["noise_floor"])
            # entry by entry on the sampled indices, against the same measure
            # between the three runs' sampled x
            fe = noise_floor_entries(o["x_sample"], [o["pairwise_x_sample"], o["fma_x_sample"]])
            ee = rel_entries(x_sample, xr)
            assert ee <= max(floor, 10 * fe), (what, key, "entries", ee, fe)
            if key == "iterations":
                for k2 in ("final_width", "deflations"):
                    if k2 in info:
                        assert info[k2] == o[k2], (what, k2, info[k2], o[k2])
            if (o["used_fallback"] == o["pairwise_used_fallback"] == o["fma_used_fallback"]
                    and "used_fallback" in info):
                assert info["used_fallback"] == o["used_fallback"], (what, info, o)
            break
    if o["status"] == 0:
        assert info["rel_res_true"] < 2 * tol, (what, info["rel_res_true"])
    return err
