"""Shared helpers of the GPU parity tests (imported by test_gpu_*.py)."""
import numpy as np
import torch

import oracle
from paper_2603_08386_amd import ddhf as D

DEV = "cuda:0"


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)


def oracle_window(win, sample=None):
    """Oracle index + active list (+ optional power of a pixel subsample)."""
    r = oracle.build_pixel_index(win.x, win.y, win.p, win.t, win.W, win.H, win.t0, win.T_w)
    act = oracle.active_pixels(r["row_ptr"], win.params.n_min)
    r["active"] = act
    return r


def power_err(P32, P64, row_ptr, active, a64):
    """max over pixels and bins of |P32 - P64| / max(P64, sum_e a_e^2)."""
    cnt = row_ptr[active + 1] - row_ptr[active]
    floor = np.zeros(active.shape[0])
    for u, q in enumerate(active):
        b, e = row_ptr[q], row_ptr[q + 1]
        floor[u] = np.sum(a64[b:e] ** 2)
    den = np.maximum(P64, floor[:, None])
    den = np.where(den > 0, den, 1.0)
    return float(np.max(np.abs(P32.astype(np.float64) - P64) / den)) if P64.size else 0.0


def gpu_window(win, **kw):
    return D.window_from_synth(win, device=DEV, **kw)


def stratified_sample(counts, k, rng, heavy_all=True):
    """Indices into counts: k spread over count deciles plus the heaviest rows."""
    order = np.argsort(counts, kind="stable")
    picks = set()
    if order.size == 0:
        return np.zeros(0, np.int64)
    for d in range(10):
        lo, hi = d * order.size // 10, (d + 1) * order.size // 10
        if hi > lo:
            picks.update(rng.choice(order[lo:hi], size=min(k // 10 + 1, hi - lo), replace=False).tolist())
    if heavy_all:
        mx = counts.max()
        picks.update(np.flatnonzero(counts == mx)[:32].tolist())
        picks.update(order[-8:].tolist())
    return np.array(sorted(picks), np.int64)
