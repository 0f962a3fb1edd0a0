"""Seeded synthetic event windows for the DDHF hot path.

This module only draws inputs: event tuples (x, y, p, t) of the kind a
temporal-contrast sensor emits (Sec. 3.1), rotor occlusion edges from the
pulse-train model (Sec. 3.2, Eq. 1-2), background clutter and noise. It holds
none of the method's arithmetic (no transform, no scoring), so both the oracle
and the device path may consume it.

Rotor model. A rotor disc of radius R centred at (cx, cy) with B = 2 blades
spinning at r rev/s occludes each disc pixel with the blade-pass frequency
f_bp = 2 r. The blade first reaches pixel p at phase phi_p, and the pixel stays
occluded for a duty fraction tau_p of every period, so every pass m gives one
OFF edge (brightness drops, polarity -1) at phi_p + m / f_bp and one ON edge
(+1) at phi_p + (m + tau_p) / f_bp. Each edge is a burst of b events with
Gaussian timestamp jitter. Timestamps are integer microseconds.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

T0_US = 1_700_000_000_000  # absolute window start; exercises the int64 path
JITTER_US = 20.0


@dataclasses.dataclass
class Grid:
    """Frequency grid f_j = f0 + j * df for j < K.

    mode 0 ("HZ"): f0, df in milli-Hertz; phase of an event at t_rel us is
    2 pi (f_j * t_rel mod 1e9) / 1e9.
    mode 1 ("MODES"): integer modes k = f0 + j * df over the window; phase is
    2 pi (k * t_rel mod T_w) / T_w.
    """
    f0: int
    df: int
    K: int
    mode: int = 0
    T_w_us: int = 0


@dataclasses.dataclass
class Params:
    """Detection hyperparameters (Table 2 symbols)."""
    tau_sf: float = 0.89
    tau_comb: float = 1.5
    alpha: float = 19.05
    eps_rel: float = 1e-6
    M: int = 4
    dk: int = 3
    h_min: int = 4
    n_min: int = 6
    a_min: int = 147


@dataclasses.dataclass
class Window:
    W: int
    H: int
    t0: int
    T_w: int
    x: np.ndarray  # uint16
    y: np.ndarray  # uint16
    p: np.ndarray  # int8, -1/+1
    t: np.ndarray  # int64 absolute microseconds, non-decreasing
    grid: Grid
    params: Params
    label: np.ndarray  # bool (H, W): union of rotor discs
    meta: Dict

    @property
    def n(self) -> int:
        return int(self.t.shape[0])


# --------------------------------------------------------------------------
# building blocks
# --------------------------------------------------------------------------

def disc_pixels(cx: int, cy: int, R: int, W: int, H: int) -> Tuple[np.ndarray, np.ndarray]:
    ys, xs = np.mgrid[-R:R + 1, -R:R + 1]
    keep = xs * xs + ys * ys <= R * R
    px = (xs[keep] + cx).astype(np.int64)
    py = (ys[keep] + cy).astype(np.int64)
    inb = (px >= 0) & (px < W) & (py >= 0) & (py < H)
    return px[inb], py[inb]


def rotor_events(rng: np.random.Generator, cx: int, cy: int, R: int, rev_hz: float,
                 T_w: int, burst: int, W: int, H: int,
                 t_start: float = 0.0) -> Tuple[np.ndarray, ...]:
    """Edge events of one two-blade rotor disc over [t_start, t_start + T_w) us.

    Returns (x, y, p, t_rel_float_us) with t relative to the window start.
    """
    px, py = disc_pixels(cx, cy, R, W, H)
    f_bp = 2.0 * rev_hz
    period = 1e6 / f_bp  # us
    psi = rng.uniform(0.0, 2.0 * math.pi)
    theta = np.arctan2(py - cy, px - cx)
    # time (us) at which a blade first reaches the pixel, mod one blade period
    phi = np.mod((theta - psi) / (2.0 * math.pi * rev_hz) * 1e6, period)
    tau = rng.uniform(0.15, 0.35, size=px.shape[0])
    m_lo = int(math.floor(t_start / period)) - 1
    m_hi = int(math.ceil((t_start + T_w) / period)) + 1
    ms = np.arange(m_lo, m_hi + 1, dtype=np.float64)
    t_off = phi[:, None] + ms[None, :] * period            # (npx, nm)
    t_on = t_off + tau[:, None] * period
    times = np.concatenate([t_off, t_on], axis=1)           # (npx, 2 nm)
    pol = np.concatenate([np.full(t_off.shape, -1, np.int8),
                          np.full(t_on.shape, 1, np.int8)], axis=1)
    xs = np.broadcast_to(px[:, None], times.shape)
    ys = np.broadcast_to(py[:, None], times.shape)
    times = np.repeat(times.ravel(), burst)
    pol = np.repeat(pol.ravel(), burst)
    xs = np.repeat(xs.ravel(), burst)
    ys = np.repeat(ys.ravel(), burst)
    times = times + rng.normal(0.0, JITTER_US, size=times.shape[0])
    keep = (times >= t_start) & (times < t_start + T_w)
    return xs[keep], ys[keep], pol[keep], times[keep]


def noise_events(rng: np.random.Generator, rate_hz: float, W: int, H: int, T_w: int,
                 t_start: float = 0.0):
    lam = rate_hz * W * H * T_w * 1e-6
    n = int(rng.poisson(lam))
    xs = rng.integers(0, W, size=n)
    ys = rng.integers(0, H, size=n)
    ts = rng.uniform(t_start, t_start + T_w, size=n)
    ps = np.where(rng.random(n) < 0.5, -1, 1).astype(np.int8)
    return xs, ys, ps, ts


def clutter_band_events(rng: np.random.Generator, W: int, H: int, T_w: int,
                        band_px: int = 40, speed_px_per_ms: float = 5.0,
                        n_edges: int = 10, per_cross: int = 1, x_start: float = -40.0):
    """A vertical band of random edges sweeping +x: every edge crossing a column
    fires per_cross events at each row of that column (non-periodic clutter)."""
    xs_l, ys_l, ps_l, ts_l = [], [], [], []
    v = speed_px_per_ms / 1000.0  # px per us
    offs = rng.uniform(0.0, band_px, size=n_edges)
    sgn = np.where(rng.random(n_edges) < 0.5, -1, 1)
    rows = np.arange(H)
    for o, s in zip(offs, sgn):
        x0 = x_start + o
        cols = np.arange(max(0, int(math.ceil(x0))), W)
        tc = (cols - x0) / v
        cols = cols[tc < T_w]
        tc = tc[tc < T_w]
        if cols.size == 0:
            continue
        cc = np.repeat(np.repeat(cols, H), per_cross)
        rr = np.repeat(np.tile(rows, cols.size), per_cross)
        tt = np.repeat(np.repeat(tc, H), per_cross)
        tt = tt + rng.normal(0.0, JITTER_US, size=tt.shape[0])
        xs_l.append(cc); ys_l.append(rr); ts_l.append(tt)
        ps_l.append(np.full(cc.shape[0], s, np.int8))
    if not xs_l:
        z = np.zeros(0)
        return z.astype(np.int64), z.astype(np.int64), z.astype(np.int8), z
    xs = np.concatenate(xs_l); ys = np.concatenate(ys_l)
    ps = np.concatenate(ps_l); ts = np.concatenate(ts_l)
    keep = (ts >= 0) & (ts < T_w)
    return xs[keep], ys[keep], ps[keep], ts[keep]


def _assemble(parts, W, H, T_w, t0, rng, time_sorted=True):
    xs = np.concatenate([q[0] for q in parts]).astype(np.int64)
    ys = np.concatenate([q[1] for q in parts]).astype(np.int64)
    ps = np.concatenate([q[2] for q in parts]).astype(np.int8)
    ts = np.rint(np.concatenate([q[3] for q in parts])).astype(np.int64)
    keep = (ts >= 0) & (ts < T_w) & (xs >= 0) & (xs < W) & (ys >= 0) & (ys < H)
    xs, ys, ps, ts = xs[keep], ys[keep], ps[keep], ts[keep]
    if time_sorted:
        order = np.argsort(ts, kind="stable")
        xs, ys, ps, ts = xs[order], ys[order], ps[order], ts[order]
    return (xs.astype(np.uint16), ys.astype(np.uint16), ps, ts + t0)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

def tiny_window(seed: int = 1) -> Window:
    """64x64 sensor, 20 ms, one drone of 4 discs (R = 4 px, 110-140 rev/s,
    blade-pass 220-280 Hz), bursts of 20 events, 2 Hz/px noise: about 40 k
    events. Grid 1-1024 Hz at 1 Hz."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W = H = 64
    T_w = 20_000
    centres = [(24, 24), (40, 24), (24, 40), (40, 40)]
    parts, label = [], np.zeros((H, W), bool)
    revs = []
    for cx, cy in centres:
        r = rng.uniform(110.0, 140.0)
        revs.append(r)
        parts.append(rotor_events(rng, cx, cy, 4, r, T_w, 20, W, H))
        px, py = disc_pixels(cx, cy, 4, W, H)
        label[py, px] = True
    parts.append(noise_events(rng, 2.0, W, H, T_w))
    x, y, p, t = _assemble(parts, W, H, T_w, T0_US, rng)
    grid = Grid(f0=1000, df=1000, K=1024, mode=0, T_w_us=T_w)
    params = Params(M=5, dk=3, h_min=3, n_min=6, tau_sf=0.89, tau_comb=1.5,
                    a_min=25, alpha=19.05)
    return Window(W, H, T0_US, T_w, x, y, p, t, grid, params, label,
                  dict(name="tiny_64x64", seed=seed, rev_hz=revs))


def medium_window(seed: int = 2, n_drones: int = 4) -> Window:
    """346x260, 50 ms: 4 drones x 4 discs (R = 5 px, blade-pass 150-400 Hz,
    two discs of each drone overlap), a 40 px clutter band sweeping at
    5 px/ms with 10 random edges, 5 Hz/px noise: about 1.5 M events.
    Grid 10-2000 Hz at 0.5 Hz (3981 bins)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W, H, T_w = 346, 260, 50_000
    parts, label = [], np.zeros((H, W), bool)
    # drone centres on a well separated lattice
    slots = [(70, 60), (270, 60), (70, 195), (270, 195)][:n_drones]
    fbp = []
    drone_boxes = []
    for (dx, dy) in slots:
        offsets = [(-8, -8), (0, -8), (-8, 8), (8, 8)]  # discs 0,1 overlap (dist 8 < 2R)
        bx = [W, H, -1, -1]
        for (ox, oy) in offsets:
            f = rng.uniform(150.0, 400.0)
            fbp.append(f)
            cx, cy = dx + ox, dy + oy
            parts.append(rotor_events(rng, cx, cy, 5, f / 2.0, T_w, 20, W, H))
            px, py = disc_pixels(cx, cy, 5, W, H)
            label[py, px] = True
            bx = [min(bx[0], px.min()), min(bx[1], py.min()), max(bx[2], px.max()),
                  max(bx[3], py.max())]
        drone_boxes.append(tuple(int(v) for v in bx))
    parts.append(clutter_band_events(rng, W, H, T_w))
    parts.append(noise_events(rng, 5.0, W, H, T_w))
    x, y, p, t = _assemble(parts, W, H, T_w, T0_US, rng)
    grid = Grid(f0=10_000, df=500, K=3981, mode=0, T_w_us=T_w)
    params = Params(M=4, dk=3, h_min=4, n_min=6, tau_sf=0.89, tau_comb=1.5,
                    a_min=49, alpha=3.0)
    return Window(W, H, T0_US, T_w, x, y, p, t, grid, params, label,
                  dict(name="medium_346x260", seed=seed, f_bp_hz=fbp,
                       drone_boxes=drone_boxes))


def _smooth_field(rng, H, W, cell=16):
    """Cheap spatially coherent random field (bilinear upsampled noise)."""
    gh, gw = H // cell + 2, W // cell + 2
    g = rng.normal(size=(gh, gw))
    yy = np.arange(H) / cell
    xx = np.arange(W) / cell
    y0 = np.floor(yy).astype(int); x0 = np.floor(xx).astype(int)
    fy = (yy - y0)[:, None]; fx = (xx - x0)[None, :]
    a = g[y0][:, x0]; b = g[y0][:, x0 + 1]
    c = g[y0 + 1][:, x0]; d = g[y0 + 1][:, x0 + 1]
    return (a * (1 - fx) + b * fx) * (1 - fy) + (c * (1 - fx) + d * fx) * fy


def _edge_crossing_times(rng, counts, theta, T_w, step_us=10.0, sigma_px_per_ms=0.5, n_dir=32):
    """Event times of an edge-crossing model under a shared random-walk camera
    motion.  The camera offset o(t) is a 2-D random walk (sigma px per sqrt(ms)
    per axis) sampled every step_us; a pixel whose local edge normal points
    along theta sees the 1-D signal s(t) = cos(theta) o_x + sin(theta) o_y and
    fires whenever its accumulated |ds| passes one more contrast step C,
    C = total |ds| over the window / count, with a random phase: polarity is
    the sign of ds at that moment.  Directions are quantised to n_dir bins, so
    pixels of similar edge direction fire in step (structured clutter, not
    white noise).  Returns (times us, polarity) in pixel-major order."""
    n_t = int(T_w / step_us)
    walk = np.cumsum(rng.normal(0.0, sigma_px_per_ms * math.sqrt(step_us / 1000.0),
                                size=(n_t, 2)), axis=0)
    tgrid = (np.arange(n_t) + 0.5) * step_us
    dbin = np.mod(np.rint(theta / (2.0 * math.pi) * n_dir).astype(np.int64), n_dir)
    ts = np.empty(int(counts.sum()))
    ps = np.empty(ts.size, np.int8)
    offs = np.concatenate([[0], np.cumsum(counts)])
    for d in range(n_dir):
        sel = np.flatnonzero(dbin == d)
        if sel.size == 0:
            continue
        a = 2.0 * math.pi * d / n_dir
        ds = np.diff(math.cos(a) * walk[:, 0] + math.sin(a) * walk[:, 1], prepend=0.0)
        tv = np.cumsum(np.abs(ds))
        total = tv[-1]
        n = counts[sel]
        phase = rng.uniform(size=sel.size)
        # event j of pixel q: accumulated |ds| reaches (j + phase_q) total / n_q
        j = np.arange(int(n.sum())) - np.repeat(np.cumsum(n) - n, n)
        levels = (j + np.repeat(phase, n)) * np.repeat(total / n, n)
        k = np.minimum(np.searchsorted(tv, levels), n_t - 1)
        dst = np.repeat(offs[sel], n) + j
        ts[dst] = tgrid[k] + rng.uniform(-0.5 * step_us, 0.5 * step_us, size=k.size)
        ps[dst] = np.where(ds[k] >= 0.0, 1, -1)
    return ts, ps


def large_window(seed: int = 3, active_frac: float = 0.60, n_heavy: int = 16,
                 heavy_count: int = 5000, clutter: str = "uniform") -> Window:
    """1280x720, 100 ms, hand-held global motion: a spatially coherent 60 %
    of pixels carry clutter events with log-normal counts (median 8,
    sigma 1.28, clipped to [1, 5000]) plus n_heavy planted pixels with exactly
    heavy_count events, and 3 drones of 4 discs.  Clutter timestamps are
    uniform in the window with random polarity (clutter="uniform", the
    fallback of the edge-crossing model), or come from the edge-crossing model
    under a random-walk camera motion of 0.5 px/ms (clutter="edges": edge
    normals from the gradient of the same smooth field).  About 10 M events.
    Grid 10-4000 Hz at 1 Hz (3991 bins)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W, H, T_w = 1280, 720, 100_000
    field = _smooth_field(rng, H, W)
    thr = np.quantile(field, 1.0 - active_frac)
    act = np.flatnonzero(field.ravel() >= thr)
    counts = np.clip(np.rint(rng.lognormal(math.log(8.0), 1.28, size=act.size)), 1, 5000).astype(np.int64)
    heavy = rng.choice(act.size, size=n_heavy, replace=False)
    counts[heavy] = heavy_count
    pix = np.repeat(act, counts)
    if clutter == "uniform":
        ts = rng.uniform(0.0, T_w, size=pix.size)
        ps = np.where(rng.random(pix.size) < 0.5, -1, 1).astype(np.int8)
    elif clutter == "edges":
        gy, gx = np.gradient(field)
        theta = np.arctan2(gy.ravel()[act], gx.ravel()[act])
        ts, ps = _edge_crossing_times(rng, counts, theta, T_w)
    else:
        raise ValueError(clutter)
    parts = [(pix % W, pix // W, ps, ts)]
    label = np.zeros((H, W), bool)
    centres = [(300, 200), (700, 450), (1050, 250)]
    fbp = []
    for (dx, dy) in centres:
        for (ox, oy) in [(-8, -8), (8, -8), (-8, 8), (8, 8)]:
            f = rng.uniform(150.0, 400.0)
            fbp.append(f)
            parts.append(rotor_events(rng, dx + ox, dy + oy, 5, f / 2.0, T_w, 20, W, H))
            px, py = disc_pixels(dx + ox, dy + oy, 5, W, H)
            label[py, px] = True
    x, y, p, t = _assemble(parts, W, H, T_w, T0_US, rng)
    grid = Grid(f0=10_000, df=1000, K=3991, mode=0, T_w_us=T_w)
    params = Params(M=4, dk=3, h_min=4, n_min=6, tau_sf=0.89, tau_comb=1.5,
                    a_min=49, alpha=3.0)
    name = "large_1280x720" if clutter == "uniform" else "large_edges_1280x720"
    return Window(W, H, T0_US, T_w, x, y, p, t, grid, params, label,
                  dict(name=name, seed=seed, f_bp_hz=fbp, n_heavy=n_heavy, clutter=clutter))


def large_edges_window(seed: int = 3) -> Window:
    """The 1280x720 window with edge-crossing clutter under random-walk motion."""
    return large_window(seed, clutter="edges")


def heavy_tail_window(seed: int = 3) -> Window:
    """The 1280x720 window with a heavier tail: 1 % of the active pixels
    (about 5,500) planted at exactly 5000 events, about 38 M events in all."""
    return large_window(seed, n_heavy=5530)


def sparse_heavy_window(seed: int = 6, n_heavy: int = 64, heavy_count: int = 5000,
                        noise_hz: float = 3.0) -> Window:
    """1280x720, 100 ms, few but very heavy pixels: n_heavy pixels with
    heavy_count uniform-time events each among sparse 3 Hz/px noise (a few
    hundred pixels reach n_min), plus the 3 drones.  The heavy pixels decide
    the NDFT time unless they are split into event chunks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W, H, T_w = 1280, 720, 100_000
    parts = [noise_events(rng, noise_hz, W, H, T_w)]
    hp = rng.choice(W * H, size=n_heavy, replace=False)
    pix = np.repeat(hp, heavy_count)
    parts.append((pix % W, pix // W, np.where(rng.random(pix.size) < 0.5, -1, 1).astype(np.int8),
                  rng.uniform(0.0, T_w, size=pix.size)))
    label = np.zeros((H, W), bool)
    for (dx, dy) in [(300, 200), (700, 450), (1050, 250)]:
        for (ox, oy) in [(-8, -8), (8, -8), (-8, 8), (8, 8)]:
            f = rng.uniform(150.0, 400.0)
            parts.append(rotor_events(rng, dx + ox, dy + oy, 5, f / 2.0, T_w, 20, W, H))
            px, py = disc_pixels(dx + ox, dy + oy, 5, W, H)
            label[py, px] = True
    x, y, p, t = _assemble(parts, W, H, T_w, T0_US, rng)
    grid = Grid(f0=10_000, df=1000, K=3991, mode=0, T_w_us=T_w)
    params = Params(M=4, dk=3, h_min=4, n_min=6, tau_sf=0.89, tau_comb=1.5,
                    a_min=49, alpha=3.0)
    return Window(W, H, T0_US, T_w, x, y, p, t, grid, params, label,
                  dict(name="sparse_heavy_1280x720", seed=seed, n_heavy=n_heavy))


def random_window(seed: int, W: int, H: int, T_w: int, n: int, grid: Grid,
                  params: Optional[Params] = None, time_sorted: bool = True,
                  polarity01: bool = False, max_t_over: int = 0) -> Window:
    """Unstructured events for edge cases: uniform pixels and times.
    max_t_over > 0 lets timestamps and coordinates spill outside the window
    and sensor so that filtering is exercised."""
    rng = np.random.Generator(np.random.PCG64(seed))
    xs = rng.integers(0, W + (2 if max_t_over else 0), size=n)
    ys = rng.integers(0, H + (2 if max_t_over else 0), size=n)
    ts = rng.integers(-max_t_over, T_w + max_t_over, size=n)
    ps = np.where(rng.random(n) < 0.5, -1, 1).astype(np.int8)
    if polarity01:
        ps = ((ps + 1) // 2).astype(np.int8)
    if time_sorted:
        o = np.argsort(ts, kind="stable")
        xs, ys, ts, ps = xs[o], ys[o], ts[o], ps[o]
    return Window(W, H, T0_US, T_w, xs.astype(np.uint16), ys.astype(np.uint16),
                  ps, ts.astype(np.int64) + T0_US, grid, params or Params(),
                  np.zeros((H, W), bool), dict(name="random", seed=seed))


def periodic_blob_window(T_w: int = 33_333, periods: int = 10, duty: float = 0.15,
                         burst: int = 3, W: int = 32, H: int = 32, x0: int = 10,
                         y0: int = 10, size: int = 3, mode_grid: bool = True,
                         noise_per_px: int = 40, seed: int = 17) -> Window:
    """A size x size blob of pixels whose occlusion edges repeat exactly
    `periods` times in a window of T_w us (period T = T_w / periods, e.g.
    3333.3 us = 300.003 Hz for a 30 FPS window): OFF bursts at
    phi_p + m T and ON bursts at phi_p + (m + duty) T, each burst event with
    N(0, 20 us) jitter, plus noise_per_px events of random polarity at uniform
    times in every blob pixel (a flat spectral floor).  mode_grid selects integer modes k = 0..63 over the
    window (0-1.9 kHz at 30 FPS); otherwise 1-1000 Hz at 1 Hz."""
    rng = np.random.Generator(np.random.PCG64(seed))
    period = T_w / periods
    xs, ys, ps, ts = [], [], [], []
    for j in range(size):
        for i in range(size):
            phi = 97.0 + 211.0 * (j * size + i)
            for m in range(-1, periods + 1):
                for t_e, pol in ((phi + m * period, -1), (phi + (m + duty) * period, 1)):
                    for _ in range(burst):
                        xs.append(x0 + i); ys.append(y0 + j); ps.append(pol)
                        ts.append(t_e + rng.normal(0.0, JITTER_US))
            for _ in range(noise_per_px):
                xs.append(x0 + i); ys.append(y0 + j)
                ps.append(1 if rng.random() < 0.5 else -1)
                ts.append(rng.uniform(0.0, T_w))
    x = np.array(xs, np.int64); y = np.array(ys, np.int64)
    t = np.rint(np.array(ts)).astype(np.int64)
    p = np.array(ps, np.int8)
    keep = (t >= 0) & (t < T_w)
    x, y, p, t = x[keep], y[keep], p[keep], t[keep]
    o = np.argsort(t, kind="stable")
    if mode_grid:
        grid = Grid(f0=0, df=1, K=64, mode=1, T_w_us=T_w)
    else:
        grid = Grid(f0=1000, df=1000, K=1000, mode=0, T_w_us=T_w)
    params = Params(M=4, dk=2, h_min=3, n_min=6, tau_sf=0.89, tau_comb=1.5, a_min=4, alpha=3.0)
    label = np.zeros((H, W), bool)
    label[y0:y0 + size, x0:x0 + size] = True
    return Window(W, H, T0_US, T_w, x[o].astype(np.uint16), y[o].astype(np.uint16), p[o],
                  t[o] + T0_US, grid, params, label,
                  dict(name="periodic_blob", f_hz=1e6 / period))


def soft_comb_batch(n_windows: int = 64, base_seed: int = 400) -> List[Window]:
    """Labelled 346x260 windows (one medium window per seed)."""
    return [medium_window(seed=base_seed + i) for i in range(n_windows)]


# --------------------------------------------------------------------------
# serving stream: 1280x720 at about 10 M events/s in 100 us packets
# --------------------------------------------------------------------------

class EventStream:
    """Continuous 1280x720 stream: 3 drones (rotor bursts of 4 events), a
    shaky-camera clutter set whose active pixels drift with a random walk
    (sigma 0.5 px/ms) and fire Poisson events, plus uniform noise. Packets
    cover [t, t + packet_us) and are time-sorted. Total rate about 10 Mev/s.
    """

    def __init__(self, seed: int = 5, W: int = 1280, H: int = 720,
                 rate_hz: float = 10e6, packet_us: int = 100,
                 drone_burst: int = 4, t_origin: int = T0_US, clutter_frac: float = 0.15,
                 noise_hz: float = 2.0):
        self.rng = np.random.Generator(np.random.PCG64(seed))
        self.W, self.H = W, H
        self.packet_us = packet_us
        self.t_origin = t_origin
        self.t_us = 0
        self.drone_burst = drone_burst
        self.rotors = []
        centres = [(int(W * fx), int(H * fy)) for fx, fy in [(0.234, 0.278), (0.547, 0.625), (0.820, 0.347)]]
        for (dx, dy) in centres:
            for (ox, oy) in [(-8, -8), (8, -8), (-8, 8), (8, 8)]:
                self.rotors.append((dx + ox, dy + oy, 5, self.rng.uniform(150.0, 400.0) / 2.0,
                                    np.random.Generator(np.random.PCG64(self.rng.integers(1 << 62)))))
        # rotor phases must be consistent across packets: draw once per rotor
        self._rotor_cache = []
        for (cx, cy, R, rev, rrng) in self.rotors:
            px, py = disc_pixels(cx, cy, R, W, H)
            f_bp = 2.0 * rev
            period = 1e6 / f_bp
            psi = rrng.uniform(0.0, 2.0 * math.pi)
            theta = np.arctan2(py - cy, px - cx)
            phi = np.mod((theta - psi) / (2.0 * math.pi * rev) * 1e6, period)
            tau = rrng.uniform(0.15, 0.35, size=px.shape[0])
            self._rotor_cache.append((px, py, period, phi, tau))
        drone_rate = sum(px.size * 2 * (1e6 / per) * drone_burst
                         for (px, _, per, _, _) in self._rotor_cache)
        self.noise_rate_px = noise_hz
        self.clutter_rate = max(rate_hz - drone_rate - self.noise_rate_px * W * H, 0.0)
        field = _smooth_field(self.rng, H + 64, W + 64)
        self.clutter_map = field >= np.quantile(field, 1.0 - clutter_frac)
        self.clutter_pix = np.flatnonzero(self.clutter_map.ravel())
        self.offset = np.zeros(2)
        self.label = np.zeros((H, W), bool)
        for (px, py, _, _, _) in self._rotor_cache:
            self.label[py, px] = True

    def next_packet(self):
        """Returns (x u16, y u16, p i8, t i64 absolute) for the next packet."""
        t_a = float(self.t_us)
        t_b = t_a + self.packet_us
        rng = self.rng
        xs_l, ys_l, ps_l, ts_l = [], [], [], []
        for (px, py, period, phi, tau) in self._rotor_cache:
            m_lo = int(math.floor((t_a - phi.max() - period) / period)) - 1
            m_hi = int(math.ceil(t_b / period)) + 1
            ms = np.arange(m_lo, m_hi + 1, dtype=np.float64)
            t_off = phi[:, None] + ms[None, :] * period
            t_on = t_off + tau[:, None] * period
            for tt, pol in ((t_off, -1), (t_on, 1)):
                tt = np.repeat(tt.ravel(), self.drone_burst)
                tt = tt + rng.normal(0.0, JITTER_US, size=tt.size)
                xx = np.repeat(np.broadcast_to(px[:, None], t_off.shape).ravel(), self.drone_burst)
                yy = np.repeat(np.broadcast_to(py[:, None], t_off.shape).ravel(), self.drone_burst)
                k = (tt >= t_a) & (tt < t_b)
                xs_l.append(xx[k]); ys_l.append(yy[k]); ts_l.append(tt[k])
                ps_l.append(np.full(int(k.sum()), pol, np.int8))
        # shaky clutter: map drifts with a random walk, sigma 0.5 px/ms
        self.offset += rng.normal(0.0, 0.5 * math.sqrt(self.packet_us / 1000.0), size=2)
        nc = int(rng.poisson(self.clutter_rate * self.packet_us * 1e-6))
        sel = self.clutter_pix[rng.integers(0, self.clutter_pix.size, size=nc)]
        cy = sel // (self.W + 64) - 32 + int(round(self.offset[1]))
        cx = sel % (self.W + 64) - 32 + int(round(self.offset[0]))
        xs_l.append(cx); ys_l.append(cy)
        ts_l.append(rng.uniform(t_a, t_b, size=nc))
        ps_l.append(np.where(rng.random(nc) < 0.5, -1, 1).astype(np.int8))
        nn = int(rng.poisson(self.noise_rate_px * self.W * self.H * self.packet_us * 1e-6))
        xs_l.append(rng.integers(0, self.W, size=nn)); ys_l.append(rng.integers(0, self.H, size=nn))
        ts_l.append(rng.uniform(t_a, t_b, size=nn))
        ps_l.append(np.where(rng.random(nn) < 0.5, -1, 1).astype(np.int8))
        xs = np.concatenate(xs_l).astype(np.int64); ys = np.concatenate(ys_l).astype(np.int64)
        ps = np.concatenate(ps_l).astype(np.int8)
        ts = np.floor(np.concatenate(ts_l)).astype(np.int64)
        keep = (xs >= 0) & (xs < self.W) & (ys >= 0) & (ys < self.H) & (ts >= self.t_us) & (ts < self.t_us + self.packet_us)
        xs, ys, ps, ts = xs[keep], ys[keep], ps[keep], ts[keep]
        o = np.argsort(ts, kind="stable")
        self.t_us += self.packet_us
        return (xs[o].astype(np.uint16), ys[o].astype(np.uint16), ps[o], ts[o] + self.t_origin)
