"""Streaming DDHF: ctypes binding of the ddhf_stream_* calls (include/ddhf.h).

A Stream owns the device state of a sliding window (per-pixel event rings,
an event log, per-pixel scores) and advances it step by step; each step can be
replayed from a captured hipGraph.  Marshalling only."""
from __future__ import annotations

import ctypes as C
from typing import List, Optional

import numpy as np
import torch

from . import ddhf as D


class StreamCfg(C.Structure):
    _fields_ = [("W", C.c_int32), ("H", C.c_int32), ("T_w_us", C.c_int64),
                ("t_origin_us", C.c_int64), ("ring_cap", C.c_int32),
                ("max_step_events", C.c_int32), ("max_touched", C.c_int32),
                ("max_boxes", C.c_int32), ("grid", D.Grid), ("params", D.Params),
                ("launch", D.Launch)]


class StreamStats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("events_accepted", C.c_int64),
                ("events_rejected", C.c_int64), ("ring_overflow", C.c_int64),
                ("touched_overflow", C.c_int64), ("n_active", C.c_int32),
                ("n_touched", C.c_int32), ("n_recomputed", C.c_int32), ("epoch_shifts", C.c_int32)]


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class Stream:
    def __init__(self, W, H, T_w_us, t_origin_us, grid, params, launch: Optional[D.Launch] = None,
                 ring_cap=64, max_step_events=32768, max_touched=32768, max_boxes=256):
        cfg = StreamCfg(W, H, T_w_us, t_origin_us, ring_cap, max_step_events, max_touched,
                        max_boxes, D.make_grid(grid), D.make_params(params),
                        launch if launch is not None else D.make_launch(D.DDHF_KERNEL_VALU, 32))
        self.cfg = cfg
        self.W, self.H = W, H
        self.max_boxes = max_boxes
        self._h = C.c_void_p()
        D._check(D.lib().ddhf_stream_create(C.byref(cfg), C.byref(self._h)), "ddhf_stream_create")
        self._boxes = (D.Box * max(max_boxes, 1))()
        self._nb = C.c_int32(0)

    def close(self):
        if self._h:
            D.lib().ddhf_stream_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def push(self, x, y, p, t):
        x = np.ascontiguousarray(x, np.uint16); y = np.ascontiguousarray(y, np.uint16)
        p = np.ascontiguousarray(p, np.int8); t = np.ascontiguousarray(t, np.int64)
        rc = D.lib().ddhf_stream_push(self._h, _np_ptr(x), _np_ptr(y), _np_ptr(p), _np_ptr(t),
                                      C.c_int32(t.shape[0]))
        D._check(rc, "ddhf_stream_push")

    def step(self, t_now_us: int, use_graph: bool = True):
        rc = D.lib().ddhf_stream_step(self._h, C.c_int64(t_now_us), C.c_int32(int(use_graph)),
                                      self._boxes, C.c_int32(self.max_boxes), C.byref(self._nb))
        # DDHF_ETRUNC: outputs are complete up to the limits (kept as a flag)
        self.truncated = rc == D.DDHF_ETRUNC
        if not self.truncated:
            D._check(rc, "ddhf_stream_step")
        n = min(self._nb.value, self.max_boxes)
        return [dict((f, getattr(b, f)) for f, _ in D.Box._fields_) for b in self._boxes[:n]], \
            self._nb.value

    def stats(self) -> dict:
        s = StreamStats()
        D._check(D.lib().ddhf_stream_stats(self._h, C.byref(s)), "ddhf_stream_stats")
        return {f: getattr(s, f) for f, _ in StreamStats._fields_}

    def scores(self, device="cuda"):
        n = self.W * self.H
        sf = torch.empty(n, dtype=torch.float32, device=device)
        snr = torch.empty(n, dtype=torch.float32, device=device)
        b = torch.empty(n, dtype=torch.int32, device=device)
        cnt = torch.empty(n, dtype=torch.int32, device=device)
        D._check(D.lib().ddhf_stream_scores(self._h, D._p(sf), D._p(snr), D._p(b), D._p(cnt)),
                 "ddhf_stream_scores")
        return sf, snr, b, cnt
