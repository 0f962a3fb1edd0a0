"""Pins of the oracle's window filter, pixel sort and CSR build (Sec. 3.5
"Event Processing") against numpy's lexsort, and of the active-pixel rule."""
import numpy as np
import pytest

import oracle
from paper_2603_08386_amd import synth
from paper_2603_08386_amd.synth import Grid


def numpy_index(w, W=None, H=None, t0=None, T_w=None, weights=None):
    W = W or w.W; H = H or w.H; t0 = w.t0 if t0 is None else t0; T_w = T_w or w.T_w
    x = w.x.astype(np.int64); y = w.y.astype(np.int64); t = w.t; p = w.p.astype(np.int64)
    ok = (t >= t0) & (t < t0 + T_w) & (x < W) & (y < H) & (p >= -1) & (p <= 1)
    idx = np.flatnonzero(ok)
    key = y[idx] * W + x[idx]
    order = np.lexsort((idx, t[idx], key))
    perm = idx[order]
    row_ptr = np.concatenate([[0], np.cumsum(np.bincount(key, minlength=W * H))]).astype(np.int32)
    a = np.where(p[perm] > 0, 1.0, -1.0)
    if weights is not None:
        a = a * weights[perm].astype(np.float64)
    return row_ptr, perm.astype(np.int32), (t[perm] - t0).astype(np.uint32), a


@pytest.mark.parametrize("kind", ["tiny", "random_unsorted", "random_spill", "pol01"])
def test_index_matches_lexsort(kind):
    if kind == "tiny":
        w = synth.tiny_window()
    elif kind == "random_unsorted":
        w = synth.random_window(5, 37, 23, 10_000, 20_000, Grid(1000, 1000, 64), time_sorted=False)
    elif kind == "random_spill":
        w = synth.random_window(6, 37, 23, 10_000, 20_000, Grid(1000, 1000, 64), max_t_over=3000)
    else:
        w = synth.random_window(7, 16, 16, 5_000, 3_000, Grid(1000, 1000, 64), polarity01=True)
    weights = np.random.default_rng(0).uniform(0.5, 2.0, size=w.n).astype(np.float32) \
        if kind == "random_unsorted" else None
    r = oracle.build_pixel_index(w.x, w.y, w.p, w.t, w.W, w.H, w.t0, w.T_w, w=weights)
    rp, perm, t_rel, a = numpy_index(w, weights=weights)
    assert np.array_equal(r["row_ptr"], rp)
    assert np.array_equal(r["perm"], perm)
    assert np.array_equal(r["t_rel"], t_rel)
    assert np.array_equal(r["a"], a)
    c = r["counters"]
    assert c[0] == w.n and c[1] == perm.shape[0]
    assert c[1] + c[2] + c[3] + c[4] == w.n
    assert c[5] == int(np.sum(np.diff(w.t) < 0))


def test_bad_polarity_counted():
    w = synth.random_window(8, 8, 8, 1000, 100, Grid(1000, 1000, 8))
    w.p[:10] = 5
    r = oracle.build_pixel_index(w.x, w.y, w.p, w.t, w.W, w.H, w.t0, w.T_w)
    assert r["counters"][4] == 10 and r["n_kept"] == 90


def test_empty_window():
    e = np.zeros(0)
    r = oracle.build_pixel_index(e.astype(np.uint16), e.astype(np.uint16), e.astype(np.int8),
                                 e.astype(np.int64), 4, 3, 0, 100)
    assert r["n_kept"] == 0 and np.all(r["row_ptr"] == 0)


def test_active_pixels_rule():
    row_ptr = np.array([0, 5, 11, 11, 17, 30], np.int32)  # counts 5, 6, 0, 6, 13
    assert list(oracle.active_pixels(row_ptr, 6)) == [1, 3, 4]
    assert list(oracle.active_pixels(row_ptr, 1)) == [0, 1, 3, 4]
    assert list(oracle.active_pixels(row_ptr, 14)) == []
