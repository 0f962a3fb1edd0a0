"""Streaming form: after each step the device state must equal a plain
recompute of the window [t_now - T_w, t_now) -- identical per-pixel event
counts and active set, scores within FP32 tolerance, masks equal except
near-threshold pixels -- and graph replay must equal direct launches.  Fault
cases (full eviction, ring overflow, out-of-order pushes) are forced from the
host and must give defined counters or statuses."""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_08386_amd import ddhf as D
from paper_2603_08386_amd import synth
from paper_2603_08386_amd.stream import Stream

from gpu_common import DEV, banner

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
        # event counts per pixel are exact
        r = oracle.build_pixel_index(win.x, win.y, win.p, win.t, 160, 120, win.t0, T_W)
        assert np.array_equal(cnt_s, np.diff(r["row_ptr"]))
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
