"""The paper's frame cadence (Sec. 3.5): a continuous event stream is cut
into consecutive, non-overlapping windows of 33,333 us (30 frames per
second), and every frame goes through the whole hot path on its own, with
Eq. 6 evaluated at integer modes k = 0..K-1 over the frame (the frame's
timestamps mapped onto [-pi, pi); the -pi offset only rotates F_k, so the
library's mode grid, phase 2 pi (k t_rel mod T_w) / T_w, gives the same
power).  Mode k is k * 1e6 / 33,333 Hz = 30.0003 k Hz.

FrameDriver only cuts host events at frame boundaries and calls the library
through ddhf.Window (argument marshalling); every step runs in the library's
kernels."""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

from . import ddhf as D
from . import synth

FRAME_US = 33_333       # 30 frames per second
MODES_K = 134           # modes 0..133: 0 to 3.98 kHz at 30 Hz spacing


def frame_grid(K: int = MODES_K, frame_us: int = FRAME_US) -> synth.Grid:
    return synth.Grid(f0=0, df=1, K=K, mode=D.DDHF_GRID_MODES, T_w_us=frame_us)


@dataclasses.dataclass
class Frame:
    index: int
    t0: int                  # absolute start (us); the frame is [t0, t0 + frame_us)
    n_events: int
    boxes: list
    n_boxes: int
    dropped: int


class FrameDriver:
    """Accumulates time-ordered host packets; each completed frame is run
    through the device path.  Frame f covers [t_origin + f T, t_origin +
    (f + 1) T) with T = frame_us."""

    def __init__(self, W: int, H: int, t_origin: int, params: synth.Params,
                 K: int = MODES_K, frame_us: int = FRAME_US, capacity: int = 1 << 20,
                 device="cuda", launch: Optional[D.Launch] = None, max_boxes: int = 256):
        self.W, self.H = int(W), int(H)
        self.frame_us = int(frame_us)
        self.grid = frame_grid(K, frame_us)
        self.params = params
        self.t_origin = int(t_origin)
        self.index = 0
        self.t_end = self.t_origin + self.frame_us
        self.capacity = int(capacity)
        self.device = device
        self.launch = launch
        self.max_boxes = max_boxes
        self._buf: List[tuple] = []
        self._win: Optional[D.Window] = None

    def push(self, x, y, p, t) -> List[Frame]:
        """Adds one packet (time ordered, and after every earlier packet);
        returns the frames it completes."""
        out = []
        t = np.asarray(t)
        while t.size and t[-1] >= self.t_end:
            k = int(np.searchsorted(t, self.t_end))
            if k:
                self._buf.append((x[:k], y[:k], p[:k], t[:k]))
            out.append(self._finish())
            x, y, p, t = x[k:], y[k:], p[k:], t[k:]
        if t.size:
            self._buf.append((x, y, p, t))
        return out

    def flush_until(self, t_now: int) -> List[Frame]:
        """Completes every frame that ends at or before t_now."""
        out = []
        while self.t_end <= t_now:
            out.append(self._finish())
        return out

    def _finish(self) -> Frame:
        if self._buf:
            xs, ys, ps, ts = (np.concatenate([b[i] for b in self._buf]) for i in range(4))
        else:
            xs = ys = np.zeros(0, np.uint16)
            ps = np.zeros(0, np.int8)
            ts = np.zeros(0, np.int64)
        self._buf = []
        t0 = self.t_end - self.frame_us
        if ts.size > self.capacity:
            raise ValueError(f"frame {self.index}: {ts.size} events exceed capacity {self.capacity}")
        if self._win is None:
            self._win = D.Window(xs, ys, ps, ts, self.W, self.H, t0, self.frame_us, self.grid,
                                 self.params, device=self.device, launch=self.launch,
                                 capacity=self.capacity, max_boxes=self.max_boxes)
        else:
            self._win.reload(xs, ys, ps, ts, t0)
        boxes, n, dropped = self._win.run()
        fr = Frame(self.index, t0, int(ts.size), boxes, n, dropped)
        self.index += 1
        self.t_end += self.frame_us
        return fr

    @property
    def window(self) -> Optional[D.Window]:
        """The device window of the last frame (its scores, mask and labels)."""
        return self._win
