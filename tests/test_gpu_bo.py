"""Bayesian optimisation of Table 2 on the device objective (F1 at IoU 0.5 of
the detected boxes against the generator's drone boxes, Sec. 4.1): a short
run must not end below its own starting points (Table 2's final values among
them), re-evaluating its best point must give the same F1, and the device
objective must agree with its box counts."""
import numpy as np
import pytest

from paper_2603_08386_amd import bo, synth

from gpu_common import DEV, banner

pytestmark = pytest.mark.gpu

T2 = dict(tau_sf=0.89, tau_comb=1.5, M=4, dk=3, h_min=4, n_min=6, a_min=147, alpha=19.05)


def test_bo_short_run_on_device_objective():
    wins = [synth.medium_window(420 + i) for i in range(2)]
    banner("bo: objective on 2 labelled windows")
    obj = bo.DetectionObjective(wins, [w.meta["drone_boxes"] for w in wins], device=DEV)
    f_t2 = obj.f1(T2)
    tp, fp, fn = obj.counts(T2)
    assert tp + fn == 8                     # 4 drones per window
    assert bo.f1_score(tp, fp, fn) == f_t2
    banner(f"  Table 2 final values: F1 {f_t2:.3f} (tp {tp}, fp {fp}, fn {fn})")
    r = bo.bayes_opt(obj, len(bo.SPACE), n_init=10, n_iter=15, seed=0, n_cand=1024,
                     x0=[bo.encode(T2)])
    banner(f"  best F1 {r.best_y:.3f} at {r.best_params}")
    assert r.y.size == 26 and r.y[0] == f_t2
    assert r.best_y >= r.y[:11].max() >= f_t2
    assert obj(r.best_x) == r.best_y         # deterministic device objective
    assert 0.0 <= r.best_y <= 1.0
