"""Width selection (the refit of the paper's Sec. 5 regression models):
the least-squares fit and the choice rule, on records with known
coefficients -- no GPU."""
import math

import numpy as np

from paper_2608_07327_amd import selector as SEL


def _records(coef_sp, coef_it, coef_pt, widths=(4, 8), count=40, seed=3):
    rng = np.random.default_rng(seed)
    recs = []
    for i in range(count):
        n = float(10 ** rng.uniform(3, 6.5))
        nnz = float(n * 10 ** rng.uniform(0.5, 1.5))
        t = float(10 ** rng.uniform(-3, 0))
        it_cg = int(10 ** rng.uniform(2, 4))
        rec = {"name": f"r{i}", "n": n, "nnz": nnz, "dense": False, "cg_seconds": t,
               "cg_iterations": it_cg, "cg_status": 0, "mbpcg": {}}
        ln, lz, lt = math.log10(n), math.log10(nnz), math.log10(t)
        for s in widths:
            c, ci, cp = coef_sp[s], coef_it[s], coef_pt[s]
            sp = 10 ** (c[0] + c[1] * ln + c[2] * lz + c[3] * lt)
            ir = ci[0] + ci[1] * ln + ci[2] * lt
            tpr = 10 ** (cp[0] + cp[1] * ln + cp[2] * lz)
            its = ir * it_cg
            rec["mbpcg"][str(s)] = {"seconds": t / sp, "iterations": its, "status": 0,
                                    "rel_res_true": 1e-9}
            # make the records self-consistent in the per-iteration ratio
            rec["mbpcg"][str(s)]["seconds"] = tpr * (t / it_cg) * its
        recs.append(rec)
    return recs


def test_fit_recovers_the_per_iteration_and_iteration_models():
    coef_sp = {4: (0.5, -0.25, 0.05, 0.13), 8: (0.9, -0.4, 0.07, 0.19)}
    coef_it = {4: (0.6, 0.02, -0.05), 8: (0.5, 0.03, -0.07)}
    coef_pt = {4: (0.13, 0.09, -0.05), 8: (-0.02, 0.2, -0.09)}
    recs = _records(coef_sp, coef_it, coef_pt)
    models = SEL.fit(recs, widths=(4, 8))
    for s in (4, 8):
        m = models[str(s)]
        it = m["iteration_ratio"]
        assert np.allclose([it["const"], it["log10_n"], it["log10_t"]], coef_it[s], atol=1e-9)
        pt = m["log10_time_per_iteration_ratio"]
        assert np.allclose([pt["const"], pt["log10_n"], pt["log10_nnz"]], coef_pt[s], atol=1e-9)
        assert it["r2"] > 0.999999 and pt["r2"] > 0.999999
        # speedup = 1 / (iteration ratio x per-iteration ratio): its fit is
        # what the data say, and predicts the records it was fitted on
        for r in recs[:5]:
            sp = r["cg_seconds"] / r["mbpcg"][str(s)]["seconds"]
            pred = SEL.predict_speedup(m, r["n"], r["nnz"], r["cg_seconds"])
            assert abs(math.log10(pred) - math.log10(sp)) < 0.5


def test_fit_skips_unconverged_pairs_and_small_samples():
    coef = {4: (0.5, -0.2, 0.05, 0.1)}
    recs = _records(coef, {4: (0.6, 0.0, 0.0)}, {4: (0.1, 0.0, 0.0)}, widths=(4,), count=6)
    for r in recs[:3]:
        r["mbpcg"]["4"]["status"] = 1
    assert SEL.fit(recs, widths=(4,)) == {}          # 3 usable pairs < 5
    recs = _records(coef, {4: (0.6, 0.0, 0.0)}, {4: (0.1, 0.0, 0.0)}, widths=(4,), count=7)
    recs[0]["mbpcg"]["4"]["rel_res_true"] = 5e-7     # reported success, missed tol
    recs[1]["cg_rel_res_true"] = 3e-8
    recs[2]["cg_rel_res_true"] = 1e-9
    assert SEL.fit(recs, widths=(4,))["4"]["samples"] == 5


def test_choose_width_prefers_cg_when_nothing_wins():
    models = {"4": {"log10_speedup": {"const": -0.3, "log10_n": 0.0, "log10_nnz": 0.0,
                                      "log10_t": 0.0}},
              "8": {"log10_speedup": {"const": -0.1, "log10_n": 0.0, "log10_nnz": 0.0,
                                      "log10_t": 0.0}}}
    assert SEL.choose_width(1e5, 1e6, 0.1, models)[0] == 1
    models["8"]["log10_speedup"]["log10_t"] = 0.5     # long CG solves favour s = 8
    s, sp = SEL.choose_width(1e5, 1e6, 10.0, models)
    assert s == 8 and sp > 1.0


def test_family_covers_every_input_kind():
    names = [name for name, _ in SEL.family()]
    for kind in ("poisson2d", "diffusion3d", "graph", "dense"):
        assert any(n.startswith(kind) for n in names)
