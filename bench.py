"""Benchmark of the DDHF hot path on one MI355X.

A step is one pass of the whole path over one resident window of events:
pixel CSR build, active list, per-pixel NDFT power, spectral flatness and
comb score, mask / components / boxes, and the box count back on the host.
Prints one JSON line (see the design doc for the fields).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 vector and FP32 matrix (dense), published
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FLOP_PER_EVENT_BIN = 8         # one complex multiply-accumulate per event and bin

WORKLOADS = {
    "large_1280x720": "large_window",
    "medium_346x260": "medium_window",
    "tiny_64x64": "tiny_window",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large_1280x720", choices=sorted(WORKLOADS))
    ap.add_argument("--kernel", default="auto", choices=["auto", "valu", "mfma"])
    ap.add_argument("--bpl", type=int, default=32)
    ap.add_argument("--split", type=int, default=0, help="split pixels with more events")
    ap.add_argument("--persistent", type=int, default=0)
    ap.add_argument("--cost-order", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle baseline sample (0 = skip)")
    return ap.parse_args()


def kernel_source_digest(names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2603_08386_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_tag, digest):
    """HBM bytes per launch measured with rocprofv3 --pmc (FETCH_SIZE, WRITE_SIZE),
    valid only while the kernel source is unchanged."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel_tag}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_digest") != digest:
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(win, target_s):
    """Oracle NDFT + flatness + comb on a uniform random sample of active pixels
    (single thread), scaled to pixel-bins per second."""
    import oracle
    r = oracle.build_pixel_index(win.x, win.y, win.p, win.t, win.W, win.H, win.t0, win.T_w)
    act = oracle.active_pixels(r["row_ptr"], win.params.n_min)
    rng = np.random.default_rng(0)
    K = win.grid.K
    done_pix, spent = 0, 0.0
    batch = 8
    order = rng.permutation(act.size)
    while spent < target_s and done_pix < act.size:
        rows = act[order[done_pix:done_pix + batch]]
        t0 = time.perf_counter()
        P = oracle.ndft_power(r["row_ptr"], r["t_rel"], r["a"], rows, win.grid)
        oracle.score_rows(P, win.grid, win.params)
        spent += time.perf_counter() - t0
        done_pix += rows.size
    return dict(value=done_pix * K / spent, unit="pixel*bins/s", cores=1, kind="oracle",
                sample=f"{done_pix} uniformly sampled active pixels of the same window "
                       f"(NDFT power + flatness + comb, FP64, one thread), {spent:.1f} s")


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU; multi-GPU runs are not part "
                                   "of it (see DESIGN.md: how the path would shard)"}))
        sys.exit(2)
    import torch
    from paper_2603_08386_amd import ddhf as D
    from paper_2603_08386_amd import synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t_gen = time.time()
    win = getattr(synth, WORKLOADS[args.workload])()
    print(f"[bench] workload {args.workload}: {win.n} events, generated in "
          f"{time.time() - t_gen:.1f}s", file=sys.stderr, flush=True)

    kernel = D.DDHF_KERNEL_VALU if args.kernel in ("auto", "valu") else D.DDHF_KERNEL_MFMA
    launch = D.make_launch(kernel, args.bpl, split_events=args.split, persistent=args.persistent)
    g = D.window_from_synth(win, device="cuda:0", launch=launch, order_by_cost=bool(args.cost_order))
    stream = torch.cuda.current_stream()
    K = int(win.grid.K)

    ev = lambda: torch.cuda.Event(enable_timing=True)
    stage_ms = {"index": [], "ndft": [], "comb": [], "detect": []}
    frame_ms = []

    def step(record):
        e0, e1, e2, e3, e4 = ev(), ev(), ev(), ev(), ev()
        t_a = time.perf_counter()
        e0.record(stream)
        g.index()
        e1.record(stream)
        na = g.fetch_n_active()
        g.alloc_spectra()
        e1b = ev(); e1b.record(stream)
        g.spectra()
        e2.record(stream)
        g.score()
        e3.record(stream)
        g.detect()
        e4.record(stream)
        nb = g.n_boxes.cpu()
        t_b = time.perf_counter()
        if record:
            stage_ms["index"].append(e0.elapsed_time(e1))
            stage_ms["ndft"].append(e1b.elapsed_time(e2))
            stage_ms["comb"].append(e2.elapsed_time(e3))
            stage_ms["detect"].append(e3.elapsed_time(e4))
            frame_ms.append((t_b - t_a) * 1e3)
        return na, int(nb[0])

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        na, nbox = step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps

    rp = g.row_ptr.cpu().numpy()
    act = g.active[:na].cpu().numpy()
    events_active = int(np.sum(rp[act + 1] - rp[act]))
    ev_bins = events_active * K
    ndft_ms = float(np.mean(stage_ms["ndft"]))
    flops = FLOP_PER_EVENT_BIN * ev_bins
    achieved_tflops = flops / (ndft_ms * 1e-3) / 1e12
    tag = "ndft_valu" if kernel == D.DDHF_KERNEL_VALU else "ndft_mfma"
    digest = kernel_source_digest(["ndft.hip", "ddhf_internal.h"])
    traffic = load_traffic(f"{tag}_{args.workload}", digest)

    out = {
        "metric": "NDFT pixel*bins/s (% FP32 VALU peak) + p50/p99 frame latency, 1280x720",
        "value": na * K / (ms_per_step * 1e-3),
        "unit": "pixel*bins/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "sensor": [win.W, win.H], "T_w_us": win.T_w,
                   "events": win.n, "active_pixels": int(na), "events_in_active": events_active,
                   "K": K, "grid_mHz": [int(win.grid.f0), int(win.grid.df)],
                   "ndft_kernel": tag, "bins_per_lane": args.bpl, "split_events": args.split,
                   "persistent": args.persistent, "cost_order": args.cost_order},
        "ndft": {"ms": ndft_ms, "pixel_bins_per_s": na * K / (ndft_ms * 1e-3),
                 "event_bins_per_s": ev_bins / (ndft_ms * 1e-3),
                 "pct_fp32_peak": 100.0 * achieved_tflops / FP32_PEAK_TFLOPS},
        "stages_ms": {k: float(np.mean(v)) for k, v in stage_ms.items()},
        "frame_latency_ms": {"p50": float(np.percentile(frame_ms, 50)),
                             "p99": float(np.percentile(frame_ms, 99)),
                             "path": "plain recompute of one 100 ms window per frame"},
        "boxes": nbox,
        "roofline": {"bound": "alu" if kernel == D.DDHF_KERNEL_VALU else "mfma",
                     "kernel": tag, "achieved": achieved_tflops, "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved_tflops / FP32_PEAK_TFLOPS,
                     "traffic": traffic},
    }
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(win, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
