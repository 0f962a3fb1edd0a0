"""Host parts of the Bayesian-optimisation tuner (Sec. 4.1, Table 2): the
search space, the box matching behind F1 at IoU 0.5, the GP surrogate and
expected improvement, and the optimiser on functions with a known maximum."""
import math

import numpy as np
import pytest

from paper_2603_08386_amd import bo


def test_space_is_table_2():
    import json, os
    here = os.path.dirname(os.path.abspath(__file__))
    t2 = json.load(open(os.path.join(here, "golden", "table2_hyperparameters.json")))
    for name, lo, hi, is_int in bo.SPACE:
        assert [lo, hi] == t2[name]["range"], name
    u = bo.encode({k: t2[k]["final"] for k in t2 if not k.startswith("_")})
    v = bo.decode(u)
    for k in v:
        assert v[k] == pytest.approx(t2[k]["final"])


def test_iou_and_matching():
    assert bo.iou((0, 0, 9, 9), (0, 0, 9, 9)) == 1.0
    assert bo.iou((0, 0, 9, 9), (10, 0, 19, 9)) == 0.0
    # 10x10 boxes overlapping in a 5x10 strip: 50 / 150
    assert bo.iou((0, 0, 9, 9), (5, 0, 14, 9)) == pytest.approx(1 / 3)
    gt = [(0, 0, 9, 9), (20, 20, 29, 29)]
    pred = [(0, 0, 9, 9), (1, 1, 10, 10), (50, 50, 60, 60)]
    # one-to-one: the exact copy takes the first truth, its near duplicate is a false positive
    assert bo.match(pred, gt) == (1, 2, 1)
    assert bo.f1_score(1, 2, 1) == pytest.approx(2 / 5)
    assert bo.match([], []) == (0, 0, 0) and bo.f1_score(0, 0, 0) == 1.0
    # IoU exactly 0.5 counts (the paper's "IoU 0.5" threshold is inclusive here)
    assert bo.match([(0, 0, 9, 9)], [(0, 0, 9, 19)]) == (1, 0, 0)


def test_gp_interpolates_and_ei_is_sound():
    rng = np.random.default_rng(0)
    X = rng.random((30, 2))
    f = lambda x: np.sin(3 * x[:, 0]) + np.cos(2 * x[:, 1])
    gp = bo.GP(2).fit(X, f(X))
    mu, sd = gp.predict(X)
    assert np.max(np.abs(mu - f(X))) < 1e-2
    Xs = rng.random((200, 2))
    mu, sd = gp.predict(Xs)
    assert np.sqrt(np.mean((mu - f(Xs)) ** 2)) < 0.05
    ei = bo.expected_improvement(mu, sd, float(f(X).max()))
    assert np.all(ei >= 0)
    # closed form at sigma -> 0: EI = max(mu - best - xi, 0)
    e0 = bo.expected_improvement(np.array([2.0, 0.5]), np.array([1e-9, 1e-9]), 1.0, xi=0.0)
    assert e0 == pytest.approx([1.0, 0.0], abs=1e-6)


def test_bayes_opt_finds_a_known_maximum():
    target = np.array([0.72, 0.31, 0.55])
    f = lambda u: -float(np.sum((np.asarray(u) - target) ** 2))
    r = bo.bayes_opt(f, 3, n_init=10, n_iter=30, seed=1, n_cand=2048)
    assert r.y.shape == (40,)
    assert np.all(np.diff(r.running_best()) >= 0)
    assert r.best_y > -2e-3                 # within ~0.03 of the optimum
    rand = max(f(np.random.default_rng(2).random(3)) for _ in range(40))
    assert r.best_y > rand
