"""The paper's cadence (Sec. 3.5): 33,333 us non-overlapping frames of the
1280x720 serving stream at integer modes k = 0..133 (Eq. 6 over the frame's
normalised timestamps), through the whole device path, against the FP64
oracle on the same frame: CSR and active list exact, flatness and comb
scores of every active pixel within FP32 tolerance, the mask equal except
within 1e-3 of a threshold, detection on the device's scores bit-exact
(boxes and their dominant frequencies k * 1e6 / T_w Hz), and every drone
found at its blade-pass frequency."""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_08386_amd import ddhf as D
from paper_2603_08386_amd import frames as F
from paper_2603_08386_amd import synth

from gpu_common import DEV, banner

pytestmark = pytest.mark.gpu

PRM = synth.Params(M=4, dk=3, h_min=4, n_min=6, tau_sf=0.89, tau_comb=1.5, a_min=49, alpha=3.0)


def test_frames_30fps_against_oracle():
    W, H = 1280, 720
    gen = synth.EventStream(seed=5, W=W, H=H, rate_hz=10e6)
    drv = F.FrameDriver(W, H, gen.t_origin, PRM, device=DEV, capacity=600_000)
    hist = []
    done = []
    banner("frames: 3 frames of the 1280x720 stream at 30 FPS")
    while len(done) < 3:
        pk = gen.next_packet()
        hist.append(pk)
        done += drv.push(*pk)
    fr = done[2]                      # the last frame the window still holds
    g = drv.window
    t0, T = fr.t0, F.FRAME_US
    xs, ys, ps, ts = (np.concatenate([h[i] for h in hist]) for i in range(4))
    keep = (ts >= t0) & (ts < t0 + T)
    r = oracle.build_pixel_index(xs[keep], ys[keep], ps[keep], ts[keep], W, H, t0, T)
    rp = r["row_ptr"]
    assert np.array_equal(g.row_ptr.cpu().numpy(), rp)
    act = oracle.active_pixels(rp, PRM.n_min)
    na = g.n_active
    act_g = g.active[:na].cpu().numpy()
    assert np.array_equal(act_g, act)
    banner(f"  frame {fr.index}: {fr.n_events} events, {na} active pixels")
    grid = F.frame_grid()
    P64 = oracle.ndft_power(rp, r["t_rel"], r["a"], act, grid)
    sf64, snr64, b64 = oracle.score_rows(P64, grid, PRM)
    sf = g.sf[:na].cpu().numpy()
    snr = g.snr[:na].cpu().numpy()
    b = g.bin[:na].cpu().numpy()
    assert np.allclose(sf, sf64, rtol=1e-3, atol=1e-6)
    assert np.allclose(snr, snr64, rtol=1e-3, atol=1e-6)
    near = (np.abs(sf64 / PRM.tau_sf - 1) <= 1e-3) | (np.abs(snr64 / PRM.tau_comb - 1) <= 1e-3)
    m64 = (sf64 <= PRM.tau_sf) & (snr64 >= PRM.tau_comb)
    mask = g.mask.cpu().numpy()[act].astype(bool)
    assert np.array_equal(mask[~near], m64[~near])
    # detection on the device's own scores: bit-exact
    tau = synth.Params(**{**PRM.__dict__})
    tau.tau_sf, tau.tau_comb = float(np.float32(PRM.tau_sf)), float(np.float32(PRM.tau_comb))
    tau.alpha = float(np.float32(PRM.alpha))
    m_o, lab_o, boxes_o, n_o = oracle.detect(act, rp, sf.astype(np.float64), snr.astype(np.float64),
                                             b, W, H, grid, tau)
    assert np.array_equal(g.mask.cpu().numpy(), m_o)
    assert np.array_equal(g.labels.cpu().numpy(), lab_o)
    assert fr.n_boxes == n_o and fr.dropped == 0
    for gb, ob in zip(fr.boxes, boxes_o):
        for k in ["x0", "y0", "x1", "y1", "n_px", "rep_pixel"]:
            assert gb[k] == ob[k]
        assert gb["f_dom_hz"] == ob["f_dom_hz"]
    # the three drones: a box over each, at a mode inside the blade-pass band
    found = 0
    for (cx, cy) in [(300, 200), (700, 450), (1050, 250)]:
        hit = [bx for bx in fr.boxes if bx["x0"] <= cx <= bx["x1"] and bx["y0"] <= cy <= bx["y1"]]
        if hit and 100.0 <= hit[0]["f_dom_hz"] <= 900.0:
            found += 1
    banner(f"  {fr.n_boxes} boxes, {found} drones at their blade-pass band")
    assert found == 3


def test_frames_cut_exactly_at_boundaries():
    """Events are assigned to [t0 + f T, t0 + (f + 1) T): the counts of every
    frame equal the host's own cut, including frames left empty."""
    W, H = 64, 48
    rng = np.random.default_rng(3)
    t_origin = synth.T0_US
    ts = np.sort(rng.integers(0, 5 * F.FRAME_US, size=20000)) + t_origin
    ts = ts[(ts < t_origin + F.FRAME_US) | (ts >= t_origin + 2 * F.FRAME_US)]   # frame 1 empty
    xs = rng.integers(0, W, size=ts.size).astype(np.uint16)
    ys = rng.integers(0, H, size=ts.size).astype(np.uint16)
    ps = np.where(rng.random(ts.size) < 0.5, -1, 1).astype(np.int8)
    drv = F.FrameDriver(W, H, t_origin, PRM, device=DEV, capacity=20000)
    out = []
    for a in range(0, ts.size, 997):
        out += drv.push(xs[a:a + 997], ys[a:a + 997], ps[a:a + 997], ts[a:a + 997])
    out += drv.flush_until(t_origin + 5 * F.FRAME_US)
    assert [f.index for f in out] == list(range(5))
    want = np.bincount((ts - t_origin) // F.FRAME_US, minlength=5)
    assert [f.n_events for f in out] == want.tolist()
    assert out[1].n_events == 0 and out[1].n_boxes == 0
