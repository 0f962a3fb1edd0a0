"""Generator checks: sizes land in each workload's stated range, labels are
the rotor discs, seeds are deterministic, and Params defaults are Table 2."""
import json
import os

import numpy as np

from paper_2603_08386_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def test_params_defaults_are_table2():
    g = json.load(open(os.path.join(HERE, "golden", "table2_hyperparameters.json")))
    p = synth.Params()
    for k, v in g.items():
        if k.startswith("_"):
            continue
        assert getattr(p, k) == v["final"], k
        assert v["range"][0] <= v["final"] <= v["range"][1]


def test_tiny_window_size_and_determinism():
    a = synth.tiny_window(1)
    b = synth.tiny_window(1)
    assert 32_000 <= a.n <= 48_000
    assert np.array_equal(a.t, b.t) and np.array_equal(a.x, b.x)
    assert np.all(np.diff(a.t) >= 0)
    assert a.t.min() >= a.t0 and a.t.max() < a.t0 + a.T_w
    assert a.label.sum() == 4 * 49
    assert set(np.unique(a.p)) <= {-1, 1}


def test_medium_window_size():
    w = synth.medium_window(2)
    assert 1.2e6 * 0.9 <= w.n <= 1.8e6
    assert w.grid.K == 3981 and w.grid.f0 + (w.grid.K - 1) * w.grid.df == 2_000_000


def test_stream_packets_are_ordered_and_bounded():
    s = synth.EventStream(seed=5)
    tot = 0
    for k in range(20):
        x, y, p, t = s.next_packet()
        assert np.all(np.diff(t) >= 0)
        assert t.min() >= s.t_origin + k * 100 and t.max() < s.t_origin + (k + 1) * 100
        assert x.max() < 1280 and y.max() < 720
        tot += t.size
    rate = tot / (20 * 100e-6)
    assert 7e6 < rate < 13e6
