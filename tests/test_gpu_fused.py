"""GPU parity of the fused spectrum + flatness + comb call (ddhf_ndft_comb,
Eq. 6-11 per pixel with the spectrum kept on chip) against the FP64 oracle
chain: events -> Eq. 6 power in FP64 -> Eq. 7 flatness and Eq. 8-11 comb in
FP64.  Bars as for the two-call path: scores within 1e-3 relative (the FP32
spectrum's error bound, |P32 - P64| <= 1e-4 max(P64, sum a^2), propagated),
the dominant bin equal wherever the oracle's top two scores differ by more
than 1e-3, the mask equal except within 1e-3 of a threshold."""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_08386_amd import ddhf as D
from paper_2603_08386_amd import synth
from paper_2603_08386_amd.synth import Grid, Params

from gpu_common import DEV, banner, oracle_window, stratified_sample
from test_gpu_parity import detect_compare, e2e_sampled, near_threshold, to_np

pytestmark = pytest.mark.gpu


def counts_window(counts, T_w, grid, params, seed=0):
    """One row of pixels, pixel i with counts[i] events at uniform random
    times (microseconds) and random polarity."""
    rng = np.random.Generator(np.random.PCG64(seed))
    counts = np.asarray(counts, np.int64)
    x = np.repeat(np.arange(counts.size), counts).astype(np.uint16)
    t = rng.integers(0, T_w, size=x.size)
    p = np.where(rng.random(x.size) < 0.5, -1, 1).astype(np.int8)
    o = np.argsort(t, kind="stable")
    x, t, p = x[o], t[o], p[o]
    return synth.Window(int(counts.size), 1, synth.T0_US, T_w, x, np.zeros_like(x), p,
                        t.astype(np.int64) + synth.T0_US, grid, params,
                        np.zeros((1, counts.size), bool), dict(name="counts", seed=seed))


def fused_scores(win, order_by_cost=True, kernel=D.DDHF_KERNEL_MFMA16):
    g = D.window_from_synth(win, device=DEV, fused=True, order_by_cost=order_by_cost,
                            launch=D.make_launch(kernel, 64))
    g.index()
    g.fetch_n_active()
    g.alloc_spectra()
    g.spectra_and_score()
    torch.cuda.synchronize()
    return g


def check_rows_against_oracle(win, g, rows=None):
    """Scores of oracle active rows `rows` (all if None) from the fused call
    against the FP64 chain; returns the number of rows compared."""
    r = oracle_window(win)
    act64 = r["active"]
    na = g.n_active
    act = to_np(g.active, na)
    order = np.argsort(act, kind="stable")
    assert np.array_equal(act[order], act64)
    if rows is None:
        rows = np.arange(act64.size)
    q = act64[rows]
    P64 = oracle.ndft_power(r["row_ptr"], r["t_rel"], r["a"], q, win.grid)
    u = order[rows]
    sf, snr, b = to_np(g.sf, na)[u], to_np(g.snr, na)[u], to_np(g.bin, na)[u]
    prm = win.params
    for i in range(rows.size):
        sf64 = oracle.spectral_flatness(P64[i], prm.eps_rel)
        s64, b64, all64 = oracle.comb_score(P64[i], win.grid, prm, want_all=True)
        assert sf[i] == pytest.approx(sf64, rel=1e-3, abs=1e-6), (q[i], sf[i], sf64)
        assert snr[i] == pytest.approx(s64, rel=1e-3, abs=1e-6), (q[i], snr[i], s64)
        top = np.sort(all64)[::-1]
        if top.size < 2 or top[0] > (1 + 1e-3) * top[1]:
            assert b[i] == b64, (q[i], b[i], b64)
    return rows.size


# pixel counts around the 256-event staging rounds and the event pairs
COUNTS = [1, 2, 3, 6, 7, 63, 64, 65, 255, 256, 257, 300, 511, 512, 513, 1001]

RAGGED = [
    # grid, params: every fast-comb specialisation and ragged K (partial last
    # tile, tiles beyond K, K below one tile)
    (Grid(f0=1000, df=1000, K=1025, mode=0), Params(M=4, dk=3, h_min=2, n_min=1)),
    (Grid(f0=5000, df=500, K=2100, mode=0), Params(M=5, dk=3, h_min=3, n_min=1)),
    (Grid(f0=10_000, df=1000, K=4096, mode=0), Params(M=4, dk=3, h_min=4, n_min=1)),
    (Grid(f0=2000, df=1000, K=37, mode=0), Params(M=3, dk=2, h_min=1, n_min=1)),
    (Grid(f0=0, df=7000, K=1000, mode=0), Params(M=6, dk=1, h_min=2, n_min=1)),
    (Grid(f0=1000, df=1000, K=5, mode=0), Params(M=1, dk=0, h_min=1, n_min=1)),
    (Grid(f0=0, df=1, K=134, mode=1, T_w_us=33_333), Params(M=4, dk=3, h_min=2, n_min=1)),
    # K a multiple of 1024 below 4096: the live waves' tiles end exactly at K
    # and the other waves hold no bins
    (Grid(f0=3000, df=1000, K=2048, mode=0), Params(M=4, dk=3, h_min=2, n_min=1)),
    (Grid(f0=2000, df=500, K=3072, mode=0), Params(M=5, dk=3, h_min=3, n_min=1)),
]


@pytest.mark.parametrize("kernel", [D.DDHF_KERNEL_MFMA16, D.DDHF_KERNEL_MFMA])
@pytest.mark.parametrize("case", range(len(RAGGED)))
def test_fused_ragged_counts_and_grids(case, kernel):
    """Split-FP16 and FP32 matrix forms of the fused kernel."""
    grid, prm = RAGGED[case]
    T_w = grid.T_w_us if grid.mode == 1 else 20_000
    win = counts_window(COUNTS, T_w, grid, prm, seed=case)
    banner(f"fused ragged K={grid.K} M={prm.M} dk={prm.dk} mode={grid.mode} kernel={kernel}")
    g = fused_scores(win, order_by_cost=bool(case % 2), kernel=kernel)
    assert check_rows_against_oracle(win, g) == len(COUNTS)


def test_fused_tiny_end_to_end():
    """64x64 window, every active pixel: scores against the FP64 chain, the
    mask equal off the thresholds, boxes equal when no pixel is near one."""
    win = synth.tiny_window(1)
    banner("fused tiny end to end")
    g = D.window_from_synth(win, device=DEV, fused=True)
    boxes, n, dropped = g.run()
    assert g.power is None  # no spectra were allocated
    check_rows_against_oracle(win, g)
    r = oracle_window(win)
    P64 = oracle.ndft_power(r["row_ptr"], r["t_rel"], r["a"], r["active"], win.grid)
    sf, snr, b = oracle.score_rows(P64, win.grid, win.params)
    m64, lab64, boxes64, n64 = oracle.detect(r["active"], r["row_ptr"], sf, snr, b, win.W, win.H,
                                             win.grid, win.params)
    amb = np.zeros(win.W * win.H, bool)
    amb[r["active"]] = near_threshold(sf, snr, win.params)
    assert np.array_equal(to_np(g.mask)[~amb], m64[~amb])
    if not amb.any():
        assert n == n64
        assert [(q["x0"], q["y0"], q["x1"], q["y1"], q["n_px"]) for q in boxes] == \
               [(q["x0"], q["y0"], q["x1"], q["y1"], q["n_px"]) for q in boxes64]
    assert n >= 1


def test_fused_medium_sampled():
    win = synth.medium_window(2)
    banner(f"fused medium n={win.n}")
    g = D.window_from_synth(win, device=DEV, fused=True, order_by_cost=True)
    boxes, n, dropped = g.run()
    torch.cuda.synchronize()
    n_rows, n_rot, n_on = e2e_sampled(win, g)
    banner(f"  {n_rows} pixels ({n_rot} rotor, {n_on} on the mask), {n} boxes")
    assert n_rot >= 100 and n_on >= 50 and n >= 1


def test_fused_mode_grid_30fps():
    """33,333 us window on integer modes: boxes and box frequency equal the
    oracle's."""
    win = synth.periodic_blob_window()
    banner("fused mode grid 30 FPS")
    g = D.window_from_synth(win, device=DEV, fused=True)
    boxes, n, dropped = g.run()
    r = oracle_window(win)
    P64 = oracle.ndft_power(r["row_ptr"], r["t_rel"], r["a"], r["active"], win.grid)
    sf, snr, b = oracle.score_rows(P64, win.grid, win.params)
    m64, lab64, boxes64, n64 = oracle.detect(r["active"], r["row_ptr"], sf, snr, b, win.W, win.H,
                                             win.grid, win.params)
    assert not near_threshold(sf, snr, win.params).any()
    assert np.array_equal(to_np(g.mask), m64) and np.array_equal(to_np(g.labels), lab64)
    assert np.array_equal(to_np(g.bin, g.n_active), b)
    assert n == n64 == 1
    assert boxes[0]["f_dom_hz"] == boxes64[0]["f_dom_hz"]


def test_fused_large_sampled_and_against_two_calls():
    """The 1280x720 window (cost-ordered, as timed): sampled pixels against the
    FP64 chain through detection; every pixel against the two-call path on the
    device (MFMA spectra to HBM, then the comb): scores within 1e-3 relative,
    and where the dominant bins differ the oracle's top two scores are within
    1e-3 of each other (a near tie either answer may take)."""
    win = synth.large_window()
    banner(f"fused large n={win.n}")
    g = D.window_from_synth(win, device=DEV, fused=True, order_by_cost=True)
    boxes, n, dropped = g.run()
    torch.cuda.synchronize()
    n_rows, n_rot, n_on = e2e_sampled(win, g, n_strat=40, n_rot=60, seed=7, n_bins=60)
    banner(f"  end to end: {n_rows} pixels ({n_rot} rotor, {n_on} on the mask), {n} boxes")
    assert n_rot >= 50 and n >= 1
    na = g.n_active
    sf_f, snr_f, b_f = to_np(g.sf, na), to_np(g.snr, na), to_np(g.bin, na)
    # the two-call path on the same index
    h = D.window_from_synth(win, device=DEV, order_by_cost=True,
                            launch=D.make_launch(D.DDHF_KERNEL_MFMA, 64))
    h.index()
    h.fetch_n_active()
    h.alloc_spectra()
    h.spectra()
    h.score()
    torch.cuda.synchronize()
    assert h.n_active == na and np.array_equal(to_np(h.active, na), to_np(g.active, na))
    sf_s, snr_s, b_s = to_np(h.sf, na), to_np(h.snr, na), to_np(h.bin, na)
    assert np.allclose(sf_f, sf_s, rtol=1e-3, atol=1e-6)
    assert np.allclose(snr_f, snr_s, rtol=1e-3, atol=1e-6)
    diff = np.flatnonzero(b_f != b_s)
    banner(f"  bins differing from the two-call path: {diff.size} of {na}")
    assert diff.size <= max(10, na // 1000)
    r = oracle_window(win)
    act = to_np(g.active, na)
    P64 = oracle.ndft_power(r["row_ptr"], r["t_rel"], r["a"], act[diff], win.grid)
    for i, u in enumerate(diff):
        _, _, all64 = oracle.comb_score(P64[i], win.grid, win.params, want_all=True)
        top = np.sort(all64)[::-1]
        assert top[0] <= (1 + 1e-3) * top[1], (act[u], b_f[u], b_s[u])
    # detection on the fused scores: exact against the oracle's detect on them
    ndet = detect_compare(act, r["row_ptr"], sf_f.astype(np.float64), snr_f.astype(np.float64),
                          b_f, win.W, win.H, win.grid, win.params)
    assert ndet >= 1


@pytest.mark.parametrize("kernel", [D.DDHF_KERNEL_MFMA16, D.DDHF_KERNEL_MFMA])
def test_fused_deterministic(kernel):
    win = synth.medium_window(2)
    g1 = fused_scores(win, kernel=kernel)
    g2 = fused_scores(win, kernel=kernel)
    na = g1.n_active
    for a, b in [(g1.sf, g2.sf), (g1.snr, g2.snr), (g1.bin, g2.bin)]:
        assert torch.equal(a[:na], b[:na])


def test_fused_unsupported_shapes_are_refused():
    win = counts_window([5, 9], 20_000, Grid(f0=1000, df=1000, K=4097, mode=0),
                        Params(n_min=1))
    g = D.window_from_synth(win, device=DEV, fused=True)
    g.index()
    g.fetch_n_active()
    g.alloc_spectra()
    with pytest.raises(D.DdhfError) as e:
        g.spectra_and_score()
    assert e.value.status == D.DDHF_EINVAL
    # a median band wider than 253 ranks (Hmax = 32 * 33 = 1056)
    win = counts_window([5, 9], 20_000, Grid(f0=1000, df=1000, K=4096, mode=0),
                        Params(M=32, dk=16, h_min=1, n_min=1))
    g = D.window_from_synth(win, device=DEV, fused=True)
    g.index()
    g.fetch_n_active()
    g.alloc_spectra()
    with pytest.raises(D.DdhfError):
        g.spectra_and_score()


def test_scoring_selector():
    """ddhf_autotune_scoring times both forms, returns positive times, and the
    window then scores with the chosen one; the scores it leaves behind equal
    the two-call path's or the fused kernel's."""
    win = synth.medium_window(2)
    g = D.window_from_synth(win, device=DEV, order_by_cost=True,
                            launch=D.make_launch(D.DDHF_KERNEL_MFMA16, 64))
    g.index()
    g.fetch_n_active()
    fused, ms_s, ms_f = g.select_scoring()
    banner(f"scoring selector: fused={fused} split {ms_s:.3f} ms fused {ms_f:.3f} ms")
    assert ms_s > 0 and ms_f > 0
    assert fused == (ms_f < 0.98 * ms_s)
    na = g.n_active
    sel = (g.sf[:na].clone(), g.snr[:na].clone(), g.bin[:na].clone())
    g.fused = False
    g.alloc_spectra()
    g.spectra_and_score()
    split = (g.sf[:na].clone(), g.snr[:na].clone(), g.bin[:na].clone())
    f = fused_scores(win)
    fz = (f.sf[:na], f.snr[:na], f.bin[:na])
    ref = fz if fused else split
    for a, b in zip(sel, ref):
        assert torch.equal(a, b)
    # a shape only the two-call path covers: the fused form is reported absent
    win2 = counts_window([5, 9, 40], 20_000, Grid(f0=1000, df=1000, K=5000, mode=0),
                         Params(n_min=1))
    h = D.window_from_synth(win2, device=DEV, launch=D.make_launch(D.DDHF_KERNEL_MFMA16, 64))
    h.index()
    h.fetch_n_active()
    fused2, ms_s2, ms_f2 = h.select_scoring()
    assert not fused2 and ms_s2 > 0 and ms_f2 == -1.0


def test_fused_weighted_events():
    """Per-event weights over twelve decades and a pixel of zero weights: the
    split-FP16 form scales each pixel's amplitudes by a power of two; scores
    against the FP64 chain."""
    rng = np.random.default_rng(21)
    grid = Grid(f0=2000, df=1000, K=1500, mode=0)
    prm = Params(M=4, dk=3, h_min=2, n_min=1)
    base = counts_window([40, 300, 7, 90, 1200, 33], 20_000, grid, prm, seed=5)
    w = (10.0 ** rng.uniform(-6, 6, size=base.n)).astype(np.float32)
    w[base.x == 2] = 0.0
    banner("fused weighted events")
    g = D.Window(base.x, base.y, base.p, base.t, base.W, base.H, base.t0, base.T_w, grid, prm,
                 w=w, device=DEV, fused=True, launch=D.make_launch(D.DDHF_KERNEL_MFMA16, 64))
    g.index()
    g.fetch_n_active()
    g.alloc_spectra()
    g.spectra_and_score()
    torch.cuda.synchronize()
    r = oracle.build_pixel_index(base.x, base.y, base.p, base.t, base.W, base.H, base.t0,
                                 base.T_w, w=w)
    act = oracle.active_pixels(r["row_ptr"], 1)
    assert np.array_equal(to_np(g.active, g.n_active), act)
    P64 = oracle.ndft_power(r["row_ptr"], r["t_rel"], r["a"], act, grid)
    sf, snr = to_np(g.sf, g.n_active), to_np(g.snr, g.n_active)
    for i in range(act.size):
        sf64 = oracle.spectral_flatness(P64[i], prm.eps_rel)
        s64, _, _ = oracle.comb_score(P64[i], grid, prm, want_all=True)
        assert sf[i] == pytest.approx(sf64, rel=1e-3, abs=1e-6), (i, sf[i], sf64)
        assert snr[i] == pytest.approx(s64, rel=1e-3, abs=1e-6), (i, snr[i], s64)
