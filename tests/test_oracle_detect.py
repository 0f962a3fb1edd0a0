"""Pins of the oracle's mask, 8-connected labelling, boxes, A_min filter and
box merge (Sec. 3.5 "Segmentation Mask Processing", Eq. 12) against
scipy.ndimage and hand-built cases."""
import numpy as np
import pytest
from scipy import ndimage

import oracle
from paper_2603_08386_amd import synth
from paper_2603_08386_amd.synth import Grid, Params

GRID = Grid(f0=10_000, df=500, K=3981)


def run_mask(mask2d, params, snr=None):
    """Drive orc_detect with every pixel active and the given mask."""
    H, W = mask2d.shape
    n = W * H
    row_ptr = (np.arange(n + 1) * 10).astype(np.int32)  # 10 events per pixel
    active = np.arange(n, dtype=np.int32)
    sf = np.where(mask2d.ravel(), 0.1, 0.99)
    s = np.where(mask2d.ravel(), 5.0, 0.0) if snr is None else snr
    b = (np.arange(n) % 100).astype(np.int32)
    return oracle.detect(active, row_ptr, sf, s, b, W, H, GRID, params)


@pytest.mark.parametrize("density", [0.05, 0.2, 0.45, 0.6])
def test_labels_and_boxes_match_scipy(density):
    rng = np.random.default_rng(int(density * 100))
    H, W = 48, 64
    m = rng.random((H, W)) < density
    prm = Params(n_min=1, tau_sf=0.5, tau_comb=1.0, a_min=1, alpha=0.0)
    mask, labels, boxes, nb = run_mask(m, prm)
    assert np.array_equal(mask.reshape(H, W).astype(bool), m)
    lab, n = ndimage.label(m, structure=np.ones((3, 3), int))
    # labels are the smallest pixel index of each component
    lab_flat = lab.ravel()
    ref = np.full(H * W, -1, np.int64)
    for c in range(1, n + 1):
        pix = np.flatnonzero(lab_flat == c)
        ref[pix] = pix.min()
    assert np.array_equal(labels, ref)
    # alpha = 0 never merges: one box per component, same bounding boxes
    objs = ndimage.find_objects(lab)
    ref_boxes = sorted((sl[0].start, sl[1].start, sl[0].stop - 1, sl[1].stop - 1,
                        int(np.sum(lab[sl] == c + 1))) for c, sl in enumerate(objs))
    got = sorted((b["y0"], b["x0"], b["y1"], b["x1"], b["n_px"]) for b in boxes)
    assert nb == n and got == ref_boxes


def blob(m, x0, y0, w, h):
    m[y0:y0 + h, x0:x0 + w] = True


def test_area_filter_keeps_area_equal_to_a_min():
    m = np.zeros((40, 40), bool)
    blob(m, 2, 2, 5, 5)    # area 25
    blob(m, 20, 20, 4, 6)  # area 24
    prm = Params(n_min=1, tau_sf=0.5, tau_comb=1.0, a_min=25, alpha=0.0)
    _, _, boxes, nb = run_mask(m, prm)
    assert nb == 1 and (boxes[0]["x0"], boxes[0]["y0"], boxes[0]["x1"], boxes[0]["y1"]) == (2, 2, 6, 6)


def test_merge_is_strict_at_alpha_times_scale():
    """Two 3x3 boxes whose centres are 6 px apart: s = 3, so alpha = 2 gives
    dist = alpha s exactly (no merge) and alpha = 2.0001 merges."""
    m = np.zeros((20, 30), bool)
    blob(m, 2, 5, 3, 3)
    blob(m, 8, 5, 3, 3)
    prm = Params(n_min=1, tau_sf=0.5, tau_comb=1.0, a_min=1, alpha=2.0)
    assert run_mask(m, prm)[3] == 2
    prm.alpha = 2.0001
    _, _, boxes, nb = run_mask(m, prm)
    assert nb == 1
    b = boxes[0]
    assert (b["x0"], b["y0"], b["x1"], b["y1"], b["n_px"]) == (2, 5, 10, 7, 18)


def test_merge_chains_transitively_and_repeats():
    """A-B and B-C are close, A-C is not: all three merge; the merged box
    then reaches D, which merges in the next round."""
    m = np.zeros((20, 80), bool)
    blob(m, 0, 8, 3, 3)    # A centre x = 1
    blob(m, 6, 8, 3, 3)    # B centre x = 7
    blob(m, 12, 8, 3, 3)   # C centre x = 13
    blob(m, 31, 8, 3, 3)   # D centre x = 32
    prm = Params(n_min=1, tau_sf=0.5, tau_comb=1.0, a_min=1, alpha=2.01)
    _, _, boxes, nb = run_mask(m, prm)
    # round 1: A,B,C -> box x 0..14 (centre 7, s = 15); D: distance 25 < 2.01 * 15
    assert nb == 1
    assert (boxes[0]["x0"], boxes[0]["x1"]) == (0, 33)


def test_representative_is_highest_score_then_lowest_index():
    m = np.zeros((10, 10), bool)
    blob(m, 2, 2, 3, 1)
    snr = np.zeros(100)
    snr[22], snr[23], snr[24] = 4.0, 7.0, 7.0
    prm = Params(n_min=1, tau_sf=0.5, tau_comb=1.0, a_min=1, alpha=0.0)
    _, _, boxes, nb = run_mask(m, prm, snr=snr)
    assert nb == 1 and boxes[0]["rep_pixel"] == 23
    assert boxes[0]["f_dom_hz"] == pytest.approx((10_000 + 23 * 500) / 1000.0)


def test_thresholds_and_n_min_gate_the_mask():
    H, W = 4, 4
    n = 16
    row_ptr = np.concatenate([[0], np.cumsum(np.full(n, 6))]).astype(np.int32)
    row_ptr[-1] = row_ptr[-2] + 5  # last pixel has 5 events
    active = np.arange(n, dtype=np.int32)
    sf = np.full(n, 0.5); sf[1] = 0.9; sf[2] = 0.89
    snr = np.full(n, 2.0); snr[3] = 1.49; snr[4] = 1.5
    b = np.zeros(n, np.int32)
    prm = Params(n_min=6, tau_sf=0.89, tau_comb=1.5, a_min=1, alpha=0.0)
    mask, _, _, _ = oracle.detect(active, row_ptr, sf, snr, b, W, H, GRID, prm)
    exp = np.ones(n, np.uint8); exp[1] = 0; exp[3] = 0; exp[15] = 0
    assert np.array_equal(mask, exp)


def test_empty_mask():
    m = np.zeros((8, 8), bool)
    prm = Params(n_min=1, tau_sf=0.5, tau_comb=1.0, a_min=1, alpha=3.0)
    mask, labels, boxes, nb = run_mask(m, prm)
    assert nb == 0 and np.all(labels == -1) and not mask.any()


def _oracle_boxes(win):
    r = oracle.build_pixel_index(win.x, win.y, win.p, win.t, win.W, win.H, win.t0, win.T_w)
    act = oracle.active_pixels(r["row_ptr"], win.params.n_min)
    P = oracle.ndft_power(r["row_ptr"], r["t_rel"], r["a"], act, win.grid)
    sf, snr, b = oracle.score_rows(P, win.grid, win.params)
    return oracle.detect(act, r["row_ptr"], sf, snr, b, win.W, win.H, win.grid, win.params), b


def test_mode_grid_box_frequency_is_the_train_frequency():
    """30 FPS window (T_w = 33,333 us) whose edges repeat exactly 10 times: on
    the mode grid the box's dominant frequency is mode 10 in Hz, 10 / 33.333 ms
    = 300.003 Hz -- the generator's own 1 / T; on the 1 Hz grid the same events
    land within a bin of it (the window's main lobe is 30 Hz wide)."""
    win = synth.periodic_blob_window()
    (mask, labels, boxes, n), b = _oracle_boxes(win)
    assert n == 1 and mask.sum() == 9
    assert np.all(b == 10)                              # mode 10 in every blob pixel
    assert boxes[0]["f_dom_hz"] == pytest.approx(win.meta["f_hz"], rel=1e-6)
    assert boxes[0]["f_dom_hz"] == pytest.approx(300.003, abs=5e-4)
    hz = synth.periodic_blob_window(mode_grid=False)
    (_, _, boxes_hz, n_hz), _ = _oracle_boxes(hz)
    assert n_hz == 1 and abs(boxes_hz[0]["f_dom_hz"] - win.meta["f_hz"]) <= 1.0


def test_mode_grid_equals_hz_grid_when_modes_are_whole_hertz():
    """At T_w = 40,000 us (25 FPS) mode k is exactly 25 k Hz, so the mode grid
    k = 0..63 and the Hz grid f = 25 k Hz give the same phases, bins and boxes,
    and both conversions to Hz give 300 Hz for a train of 12 periods."""
    mode = synth.periodic_blob_window(T_w=40_000, periods=12)
    hz = synth.periodic_blob_window(T_w=40_000, periods=12)
    hz.grid = Grid(f0=0, df=25_000, K=64, mode=0, T_w_us=40_000)
    (m1, l1, b1, n1), bins1 = _oracle_boxes(mode)
    (m2, l2, b2, n2), bins2 = _oracle_boxes(hz)
    assert np.array_equal(bins1, bins2) and np.all(bins1 == 12)
    assert np.array_equal(m1, m2) and n1 == n2 == 1
    assert b1 == b2 and b1[0]["f_dom_hz"] == 300.0
