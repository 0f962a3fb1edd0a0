"""Streaming form: after each step the device state must equal the FP64
oracle on the window [t_now - T_w, t_now) -- identical per-pixel event counts,
power within the NDFT bound, flatness and comb scores within FP32 tolerance,
mask bits equal except near-threshold pixels -- and the plain device path of
the same window; graph replay must equal direct launches; moving the epoch
(32-bit stored times) must leave every result bit-identical.  Fault cases (full
eviction, ring overflow, out-of-order pushes, a window end too far past the
epoch) are forced from the host and must give defined counters or statuses."""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_08386_amd import ddhf as D
from paper_2603_08386_amd import synth
from paper_2603_08386_amd.stream import Stream

from gpu_common import DEV, banner, stratified_sample

pytestmark = pytest.mark.gpu

GRID = synth.Grid(f0=10_000, df=1000, K=1991)        # 10-2000 Hz at 1 Hz
PRM = synth.Params(M=4, dk=3, h_min=4, n_min=6, tau_sf=0.89, tau_comb=1.5, a_min=25, alpha=3.0)
T_W = 20_000


def make_stream(**kw):
    args = dict(W=160, H=120, T_w_us=T_W, t_origin_us=synth.T0_US, grid=GRID, params=PRM,
                ring_cap=128, max_step_events=8192, max_touched=8192, max_boxes=128)
    args.update(kw)
    return Stream(**args)


def plain_window(xs, ys, ps, ts, t_now):
    keep = (ts >= t_now - T_W) & (ts < t_now)
    return synth.Window(160, 120, t_now - T_W, T_W, xs[keep], ys[keep], ps[keep], ts[keep], GRID,
                        PRM, np.zeros((120, 160), bool), {})


def drive(st, gen, n_steps, packets_per_step=10, use_graph=True, hist=None):
    for _ in range(n_steps):
        for _ in range(packets_per_step):
            x, y, p, t = gen.next_packet()
            st.push(x, y, p, t)
            if hist is not None:
                hist.append((x, y, p, t))
        boxes, nb = st.step(gen.t_origin + gen.t_us, use_graph=use_graph)
    return boxes, nb


def cat(hist):
    return [np.concatenate([h[i] for h in hist]) for i in range(4)]


def oracle_check(st, hist, t_now, W, H, T_w, grid, prm, label, n_other, seed):
    """Stream state against the FP64 oracle on the window [t_now - T_w, t_now):
    counts of every pixel exact; on every labelled (rotor) active pixel up to
    n_other, plus n_other stratified other active pixels: oracle NDFT (Eq. 6) ->
    flatness and comb (Eq. 7-11) vs the stream's scores, and the mask bit
    (count >= n_min, SF <= tau_sf, SNR >= tau_comb) equal except within 1e-3 of
    a threshold.  Returns (sampled rows, rotor rows)."""
    xs, ys, ps, ts = cat(hist)
    keep = (ts >= t_now - T_w) & (ts < t_now)
    r = oracle.build_pixel_index(xs[keep], ys[keep], ps[keep], ts[keep], W, H, t_now - T_w, T_w)
    sf_s, snr_s, bin_s, cnt_s = (v.cpu().numpy() for v in st.scores())
    rp = r["row_ptr"]
    assert np.array_equal(cnt_s, np.diff(rp))
    act = oracle.active_pixels(rp, prm.n_min)
    assert act.size > 0
    rng = np.random.default_rng(seed)
    lab = label.ravel()[act]
    rot = np.flatnonzero(lab)
    if rot.size > n_other:
        rot = np.sort(rng.choice(rot, n_other, replace=False))
    counts = rp[act + 1] - rp[act]
    oth = np.flatnonzero(~lab)
    oth = oth[stratified_sample(counts[oth], n_other, rng)] if oth.size else oth
    rows = np.unique(np.concatenate([rot, oth]))
    q = act[rows]
    P64 = oracle.ndft_power(rp, r["t_rel"], r["a"], q, grid)
    sf64, snr64, b64 = oracle.score_rows(P64, grid, prm)
    assert np.allclose(sf_s[q], sf64, rtol=1e-3, atol=1e-6)
    assert np.allclose(snr_s[q], snr64, rtol=1e-3, atol=1e-6)
    near = (np.abs(sf64 / prm.tau_sf - 1) <= 1e-3) | (np.abs(snr64 / prm.tau_comb - 1) <= 1e-3)
    m_s = (sf_s[q] <= np.float32(prm.tau_sf)) & (snr_s[q] >= np.float32(prm.tau_comb))
    m_64 = (sf64 <= prm.tau_sf) & (snr64 >= prm.tau_comb)
    assert np.array_equal(m_s[~near], m_64[~near])
    # dominant bin (its frequency f0 + bin df) wherever the oracle's two best
    # candidates differ by more than 1e-3
    for i in range(min(rows.size, 160)):
        s64, bb64, all64 = oracle.comb_score(P64[i], grid, prm, want_all=True)
        assert bb64 == b64[i]
        top = np.sort(all64)[::-1]
        if top.size < 2 or top[0] > (1 + 1e-3) * top[1]:
            assert bin_s[q[i]] == bb64, (q[i], bin_s[q[i]], bb64)
    return rows, rot


@pytest.mark.parametrize("use_graph", [True, False])
def test_stream_equals_plain_recompute(use_graph):
    gen = synth.EventStream(seed=11, W=160, H=120, rate_hz=2e6)
    st = make_stream()
    hist = []
    banner(f"stream vs plain use_graph={use_graph}")
    for check in range(3):
        boxes, nb = drive(st, gen, 12, use_graph=use_graph, hist=hist)
        t_now = gen.t_origin + gen.t_us
        xs, ys, ps, ts = cat(hist)
        win = plain_window(xs, ys, ps, ts, t_now)
        sf_s, snr_s, bin_s, cnt_s = (v.cpu().numpy() for v in st.scores())
        # counts exact; sampled pixels (all rotor pixels) against the FP64 oracle
        oracle_check(st, hist, t_now, 160, 120, T_W, GRID, PRM, gen.label, n_other=80,
                     seed=check)
        # plain device path on the same window
        g = D.window_from_synth(win, device=DEV)
        pboxes, pn, _ = g.run()
        act = g.active[:g.n_active].cpu().numpy()
        sf_p = g.sf[:g.n_active].cpu().numpy()
        snr_p = g.snr[:g.n_active].cpu().numpy()
        assert np.allclose(sf_s[act], sf_p, rtol=1e-3, atol=1e-6)
        assert np.allclose(snr_s[act], snr_p, rtol=1e-3, atol=1e-6)
        near = (np.abs(sf_p / PRM.tau_sf - 1) <= 1e-3) | (np.abs(snr_p / PRM.tau_comb - 1) <= 1e-3)
        m_s = (sf_s[act] <= np.float32(PRM.tau_sf)) & (snr_s[act] >= np.float32(PRM.tau_comb))
        m_p = (sf_p <= np.float32(PRM.tau_sf)) & (snr_p >= np.float32(PRM.tau_comb))
        assert np.array_equal(m_s[~near], m_p[~near])
        if not near.any():
            assert nb == pn
            assert [(b["x0"], b["y0"], b["x1"], b["y1"]) for b in boxes] == \
                   [(b["x0"], b["y0"], b["x1"], b["y1"]) for b in pboxes[:len(boxes)]]
    s = st.stats()
    assert s["ring_overflow"] == 0 and s["touched_overflow"] == 0
    assert s["steps"] == 36
    st.close()


def test_stream_graph_replay_matches_direct():
    out = []
    for use_graph in (True, False):
        gen = synth.EventStream(seed=12, W=160, H=120, rate_hz=2e6)
        st = make_stream()
        drive(st, gen, 30, use_graph=use_graph)
        out.append([v.cpu().numpy() for v in st.scores()])
        st.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_stream_full_eviction_on_time_jump():
    gen = synth.EventStream(seed=13, W=160, H=120, rate_hz=1e6)
    st = make_stream()
    drive(st, gen, 25)
    assert st.stats()["n_active"] > 0
    t_jump = gen.t_origin + gen.t_us + 10 * T_W
    boxes, nb = st.step(t_jump)
    assert nb == 0
    _, _, _, cnt = st.scores()
    assert int(cnt.sum().item()) == 0
    assert st.stats()["n_active"] == 0
    st.close()


def test_stream_ring_overflow_is_counted():
    st = make_stream(ring_cap=4)
    t0 = synth.T0_US + 1000
    n = 10
    st.push(np.full(n, 5, np.uint16), np.full(n, 7, np.uint16), np.ones(n, np.int8),
            t0 + np.arange(n, dtype=np.int64))
    st.step(t0 + 100)
    s = st.stats()
    assert s["ring_overflow"] == n - 4
    _, _, _, cnt = st.scores()
    assert int(cnt[7 * 160 + 5].item()) == 4
    st.close()


def test_stream_rejects_bad_input():
    st = make_stream()
    t0 = synth.T0_US + 5000
    with pytest.raises(D.DdhfError):  # out of order inside a packet
        st.push(np.zeros(2, np.uint16), np.zeros(2, np.uint16), np.ones(2, np.int8),
                np.array([t0 + 5, t0 + 1], np.int64))
    st.push(np.array([3, 500], np.uint16), np.array([3, 3], np.uint16), np.array([1, 1], np.int8),
            np.array([t0, t0 + 1], np.int64))  # x = 500 is outside the sensor
    with pytest.raises(D.DdhfError):  # older than what was pushed
        st.push(np.zeros(1, np.uint16), np.zeros(1, np.uint16), np.ones(1, np.int8),
                np.array([t0 - 10], np.int64))
    st.step(t0 + 10)
    s = st.stats()
    assert s["events_rejected"] == 1 and s["events_accepted"] == 1
    # an empty step is fine
    boxes, nb = st.step(t0 + 20)
    assert nb == 0
    st.close()


# ---------------------------------------------------------------------------
# serving shape: 1280x720, ~10 Mev/s, 50 ms window, 1 ms step, against the oracle
# ---------------------------------------------------------------------------

C5_GRID = synth.Grid(f0=10_000, df=1000, K=3991)   # 10-4000 Hz at 1 Hz
C5_PRM = synth.Params(M=4, dk=3, h_min=4, n_min=6, tau_sf=0.89, tau_comb=1.5, a_min=49,
                      alpha=3.0)


def test_stream_serving_shape_against_oracle():
    W, H, T_w = 1280, 720, 50_000
    gen = synth.EventStream(seed=5, W=W, H=H, rate_hz=10e6)
    st = Stream(W, H, T_w, gen.t_origin, C5_GRID, C5_PRM,
                launch=D.make_launch(D.DDHF_KERNEL_MFMA, 64), ring_cap=256,
                max_step_events=32768, max_touched=32768, max_boxes=256)
    hist = []
    banner("stream 1280x720 10 Mev/s against the oracle")
    checked = 0
    for k, n_steps in enumerate((55, 12)):
        drive(st, gen, n_steps, hist=hist)
        t_now = gen.t_origin + gen.t_us
        rows, rot = oracle_check(st, hist, t_now, W, H, T_w, C5_GRID, C5_PRM, gen.label,
                                 n_other=120, seed=k)
        banner(f"  step {len(hist) // 10}: {rows.size} pixels checked ({rot.size} rotor)")
        assert rot.size >= 50
        checked += rows.size
        # keep the history to the window
        hist = [h for h in hist if h[3].size and h[3][-1] >= t_now - T_w]
    s = st.stats()
    assert s["ring_overflow"] == 0 and s["touched_overflow"] == 0
    assert s["events_accepted"] > 600_000
    st.close()


# ---------------------------------------------------------------------------
# 32-bit stored times: epoch shifts by whole grid periods
# ---------------------------------------------------------------------------

T_PER = 1_000_000   # 1e9 / gcd(1e9, 10000, 1000) us for GRID


def test_stream_epoch_shift_is_bit_exact():
    """Stream B's epoch lies 2147 s (a whole number of grid periods) before
    stream A's; B passes 2^31 us after its epoch 26 steps in, with a full
    window stored, and moves its epoch.  Every step's scores and boxes equal
    A's bit for bit, before and after the shift, and B still matches the
    oracle afterwards."""
    start = synth.T0_US + 458_000
    gens = [synth.EventStream(seed=14, W=160, H=120, rate_hz=2e6, t_origin=start)
            for _ in range(2)]
    a = make_stream(t_origin_us=synth.T0_US)
    b = make_stream(t_origin_us=synth.T0_US - 2147 * T_PER)
    hist = []
    banner("stream epoch shift")
    for step in range(40):
        out = []
        for st, gen in ((a, gens[0]), (b, gens[1])):
            out.append(drive(st, gen, 1, hist=hist if st is a else None))
        assert out[0] == out[1]
        sa = [v.cpu().numpy() for v in a.scores()]
        sb = [v.cpu().numpy() for v in b.scores()]
        for u, v in zip(sa, sb):
            assert np.array_equal(u, v), step
    assert a.stats()["epoch_shifts"] == 0
    assert b.stats()["epoch_shifts"] == 1
    t_now = start + gens[1].t_us
    oracle_check(b, hist, t_now, 160, 120, T_W, GRID, PRM, gens[1].label, n_other=60, seed=3)
    a.close()
    b.close()


def test_stream_first_window_near_2_32_us_past_epoch():
    """The first window ends 3 ms before 2^32 us past the epoch (the epoch is
    not a whole number of grid periods before the events): the epoch moves at
    the first step and the state matches the oracle and a stream whose epoch
    is the start of the events."""
    start = synth.T0_US + 7_000
    gens = [synth.EventStream(seed=15, W=160, H=120, rate_hz=2e6, t_origin=start)
            for _ in range(2)]
    a = make_stream(t_origin_us=start)
    c = make_stream(t_origin_us=start + 1000 - ((1 << 32) - 3000))
    hist = []
    banner("stream first window near 2^32 us")
    for step in range(30):
        drive(a, gens[0], 1, hist=hist)
        drive(c, gens[1], 1)
    assert c.stats()["epoch_shifts"] == 1
    sa = [v.cpu().numpy() for v in a.scores()]
    sc = [v.cpu().numpy() for v in c.scores()]
    assert np.array_equal(sa[3], sc[3])  # counts
    act = sa[3] >= PRM.n_min
    assert np.allclose(sa[0][act], sc[0][act], rtol=1e-3, atol=1e-6)
    assert np.allclose(sa[1][act], sc[1][act], rtol=1e-3, atol=1e-6)
    t_now = start + gens[1].t_us
    oracle_check(c, hist, t_now, 160, 120, T_W, GRID, PRM, gens[1].label, n_other=60, seed=4)
    a.close()
    c.close()


def test_stream_step_too_far_past_epoch_is_refused():
    st = make_stream(t_origin_us=synth.T0_US)
    t0 = synth.T0_US + 1000
    st.push(np.array([3], np.uint16), np.array([3], np.uint16), np.array([1], np.int8),
            np.array([t0], np.int64))
    st.step(t0 + 10)
    with pytest.raises(D.DdhfError):   # window end 2^32 us past the epoch, gap > 2^31 us
        st.step(synth.T0_US + (1 << 32) + 5000)
    with pytest.raises(D.DdhfError):   # window end before the previous one
        st.step(t0 + 5)
    boxes, nb = st.step(t0 + 20)       # the stream is still usable
    assert nb == 0
    st.close()


def test_stream_step_reports_truncation():
    """A frame with more boxes than the caller's limit: DDHF_ETRUNC after every
    output is written (true count reported, no box copied past the limit)."""
    gen = synth.EventStream(seed=16, W=160, H=120, rate_hz=2e6)
    st = make_stream(max_boxes=0)
    banner("stream truncation")
    boxes, nb = drive(st, gen, 30)
    assert nb >= 1 and boxes == [] and st.truncated
    st.close()
    st = make_stream()
    gen = synth.EventStream(seed=16, W=160, H=120, rate_hz=2e6)
    boxes, nb2 = drive(st, gen, 30)
    assert nb2 == nb and len(boxes) == nb and not st.truncated
    st.close()
