"""Shared pieces of the golden-file writers: the oracle in its three rounding
variants (reference, blocked-pairwise sums, fused multiply-adds) and the
record kept per solve.  Only the oracle and the input generators are used.
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402

VARIANTS = O.VARIANTS


def run_variant(variant, fn, *a, **kw):
    """fn(*a, **kw) under one rounding variant (the reference afterwards)."""
    O.set_variant(variant)
    try:
        return fn(*a, **kw)
    finally:
        O.set_variant("seq")


def noise_floor(xs):
    """Largest relative distance between two of the variants' solutions."""
    nb = float(np.linalg.norm(xs[0]))
    if nb == 0.0:
        return 0.0
    return max(float(np.linalg.norm(a - c)) / nb for k, a in enumerate(xs) for c in xs[k + 1:])


def mbpcg_record(runs, idx, **extra):
    """runs: {variant: (x, info)} for the three variants.  The reference run's
    diagnostics, the other variants' counts and fallback choices, the noise
    floor, |x| and x at the indices idx."""
    x0, i0 = runs["seq"]
    rec = dict(extra)
    rec.update({
        "iterations": i0["iterations"], "status": i0["status"],
        "best_column": i0["best_column"], "final_width": i0["final_width"],
        "deflations": i0["deflations"], "used_fallback": i0["used_fallback"],
        "rel_res_best": i0["rel_res_best"], "rel_res_ls": i0["rel_res_ls"],
        "rel_res_true": i0["rel_res_true"], "ls_kept": i0.get("ls_kept"),
        "seconds": i0["seconds"],
        "pairwise_iterations": runs["pairwise"][1]["iterations"],
        "fma_iterations": runs["fma"][1]["iterations"],
        "pairwise_used_fallback": runs["pairwise"][1]["used_fallback"],
        "fma_used_fallback": runs["fma"][1]["used_fallback"],
        "noise_floor": noise_floor([runs[v][0] for v in VARIANTS]),
        "x_norm": float(np.linalg.norm(x0)),
        "x_sample": np.asarray(x0)[idx].tolist(),
    })
    # the other variants' samples, for a GPU run that matches their count
    for v in VARIANTS[1:]:
        rec[f"{v}_x_sample"] = np.asarray(runs[v][0])[idx].tolist()
    return rec
