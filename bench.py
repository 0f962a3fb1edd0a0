"""Benchmark of the DDHF hot path on one MI355X.

Window leg (the step): one pass of the whole path over one resident
1280x720, 100 ms window of about 11 M events -- pixel CSR build, active list,
per-pixel NDFT power, spectral flatness and comb score, mask / components /
boxes, and the box count back on the host.  `value` is active pixels x bins
per second of the whole step; the `ndft` block and `roofline` are for the NDFT
kernel alone (HIP events on its launch stream).

Stream leg: a continuous 1280x720 stream at about 10 M events/s in 100 us
packets, 50 ms sliding window advanced every 1 ms; frame latency is measured
on the host from the push of a step's last packet to its boxes being readable,
for the graph-replayed streaming step and for a plain recompute of the window
(events copied to the device, whole path, boxes back).

Prints one JSON line.
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
FP16_PEAK_TFLOPS = 2500.0      # MI355X FP16 matrix (dense), published
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FLOP_PER_EVENT_BIN = 8         # one complex multiply-accumulate per event and bin
SOFT_FLOP_PER_EVENT_HARMONIC = 16  # forward complex MAC (8) + backward Re/Im of conj(F) z (8)

WORKLOADS = {
    "large_1280x720": "large_window",
    "large_edges_1280x720": "large_edges_window",
    "heavy_tail_1280x720": "heavy_tail_window",
    "sparse_heavy_1280x720": "sparse_heavy_window",
    "medium_346x260": "medium_window",
    "tiny_64x64": "tiny_window",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large_1280x720", choices=sorted(WORKLOADS))
    ap.add_argument("--kernel", default="auto", choices=["auto", "valu", "mfma", "mfma16"])
    ap.add_argument("--scoring", default="auto", choices=["auto", "split", "fused"],
                    help="spectra to HBM then comb, the fused spectrum + comb kernel, or the "
                         "faster of the two on this window (ddhf_autotune_scoring)")
    ap.add_argument("--bpl", type=int, default=64)
    ap.add_argument("--split", type=int, default=0, help="split pixels with more events")
    ap.add_argument("--persistent", type=int, default=0)
    ap.add_argument("--nufft", type=int, default=0,
                    help="pixels with at least this many events take the NUFFT path (0 = never)")
    ap.add_argument("--cost-order", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="target CPU time of the oracle baseline sample (0 = skip)")
    ap.add_argument("--stream-steps", type=int, default=10000,
                    help="timed stream steps (0 = skip)")
    ap.add_argument("--stream-warmup", type=int, default=500, help="untimed stream steps")
    ap.add_argument("--plain-frames", type=int, default=200, help="plain recompute frames timed")
    ap.add_argument("--cadence-frames", type=int, default=300,
                    help="33,333 us frames of the 30 FPS leg (0 = skip)")
    ap.add_argument("--soft-windows", type=int, default=64,
                    help="346x260 labelled windows in the soft-comb training leg (0 = skip)")
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="processes of the all-cores oracle baseline (capped at the CPU count)")
    ap.add_argument("--soft-steps", type=int, default=10, help="timed soft-comb training steps")
    ap.add_argument("--autotune-cache", default=None,
                    help="JSON-lines autotuner cache: read the launch from it, or time the "
                         "candidates and append the winner (default: always time)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of COPY_BYTES (the known-size kernel "
                         "that FETCH_SIZE / WRITE_SIZE are scaled by) and exit")
    ap.add_argument("--counter-summary", nargs="+", metavar="CSV",
                    help="print per-dispatch means of every rocprofv3 --pmc counter in these "
                         "counter_collection.csv files for the NDFT and comb kernels, with "
                         "derived per-wave and utilisation figures, then exit")
    ap.add_argument("--traffic-summary", nargs=4,
                    metavar=("FETCH_CSV", "WRITE_CSV", "CAL_FETCH_CSV", "CAL_WRITE_CSV"),
                    help="write profiles/traffic_<kernel>_<workload>.json from rocprofv3 --pmc "
                         "counter CSVs of this bench (--kernel valu|mfma) and of "
                         "--copy-calibration, then exit")
    return ap.parse_args()


COPY_BYTES = 256 << 20


def copy_calibration():
    import torch
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES, "launches": 3}), flush=True)


def _pmc_mean_kib(path, counter, name_part, required=True):
    """Mean per-dispatch value of one counter over the dispatches whose kernel
    name contains name_part (rocprofv3 counter_collection.csv); (None, 0) when
    there are none and required is False."""
    import csv
    vals = []
    with open(path) as f:
        for r in csv.DictReader(f):
            parts = (name_part,) if isinstance(name_part, str) else name_part
            if r["Counter_Name"] == counter and all(q in r["Kernel_Name"] for q in parts):
                vals.append(float(r["Counter_Value"]))
    if not vals:
        if not required:
            return None, 0
        raise SystemExit(f"no {counter} rows for kernels named *{name_part}* in {path}")
    return sum(vals) / len(vals), len(vals)


# sources whose digest keys a traffic record
TRAFFIC_SOURCES = {"ndft": ["ndft.hip", "phase.h", "ddhf_internal.h"],
                   "comb": ["comb.hip", "phase.h", "ddhf_internal.h"]}


KERNEL_NAMES = {0: "valu", 1: "mfma", 2: "mfma16"}


def ndft_tag(kernel, bpl):
    """Record tag and rocprofv3 kernel-name fragment of one NDFT instantiation."""
    if kernel == "mfma":
        return f"ndft_mfma{bpl}", f"k_ndft_mfma<{bpl // 16}, 0>"
    if kernel == "mfma16":
        return f"ndft_mfma16_{bpl}", f"k_ndft_mfma16<{bpl // 16}, 0>"
    return f"ndft_valu{bpl}", f"k_ndft_valu<{bpl}, 0>"


def fused_tag(kernel):
    """Record tag and rocprofv3 kernel-name fragment of the fused spectrum +
    comb kernel: its split-FP16 form unless the launch asks for the FP32
    matrix kernel."""
    if kernel == "mfma":
        return "ndft_comb_mfma", ("k_ndft_comb<", ", false>")
    return "ndft_comb_mfma16", ("k_ndft_comb<", ", true>")


def traffic_summary(args, fetch_csv, write_csv, cal_fetch_csv, cal_write_csv, out_dir=None):
    """HBM bytes per launch of the NDFT kernel and of the comb kernel, or of the
    fused kernel, whichever the profiled run launched: FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch), each scaled by bytes / reading of the plain
    copy kernel."""
    if args.kernel not in ("valu", "mfma", "mfma16"):
        raise SystemExit("--traffic-summary needs --kernel valu, mfma or mfma16")
    cf, _ = _pmc_mean_kib(cal_fetch_csv, "FETCH_SIZE", "copyBuffer")
    cw, _ = _pmc_mean_kib(cal_write_csv, "WRITE_SIZE", "copyBuffer")
    fetch_scale = COPY_BYTES / (cf * 1024.0)
    write_scale = COPY_BYTES / (cw * 1024.0)
    ntag, nname = ndft_tag(args.kernel, args.bpl)
    ftag, fname = fused_tag(args.kernel)
    found = 0
    for prefix, name, srcs in ((ntag, nname, TRAFFIC_SOURCES["ndft"]),
                               ("comb_fast", "k_comb_fast<", TRAFFIC_SOURCES["comb"]),
                               (ftag, fname, TRAFFIC_SOURCES["comb"])):
        f, nf = _pmc_mean_kib(fetch_csv, "FETCH_SIZE", name, required=False)
        w, nw = _pmc_mean_kib(write_csv, "WRITE_SIZE", name, required=False)
        if not nf or not nw:
            continue
        found += 1
        rec = {"kernel": name if isinstance(name, str) else "*".join(name),
               "workload": args.workload,
               "source_digest": kernel_source_digest(srcs),
               "fetch_kib_per_dispatch": f, "write_kib_per_dispatch": w, "dispatches": [nf, nw],
               "copy_fetch_kib": cf, "copy_write_kib": cw,
               "fetch_scale": fetch_scale, "write_scale": write_scale,
               "bytes_per_launch": f * 1024.0 * fetch_scale + w * 1024.0 * write_scale}
        out = os.path.join(out_dir or os.path.join(ROOT, "profiles"),
                           f"traffic_{prefix}_{args.workload}.json")
        with open(out, "w") as fo:
            json.dump(rec, fo, indent=1)
            fo.write("\n")
        print(json.dumps(rec), flush=True)
    if not found:
        raise SystemExit(f"no FETCH_SIZE / WRITE_SIZE rows for {nname}, k_comb_fast or "
                         f"{fname} in {fetch_csv}, {write_csv}")


MI355X_CUS, MI355X_SIMDS, MI355X_XCDS = 256, 1024, 8


def counter_summary(paths):
    """Means per dispatch of each counter for the kernels of the step, and the
    figures derived from them: VALU / LDS / SALU instructions per wave,
    VALUBusy = SQ_ACTIVE_INST_VALU (quad-cycles summed over SIMDs) / CUs /
    GRBM_GUI_ACTIVE of one XCD, MfmaUtil = SQ_VALU_MFMA_BUSY_CYCLES / SIMDs /
    GRBM_GUI_ACTIVE of one XCD (rocprofv3's own definitions; GRBM_GUI_ACTIVE
    is reported summed over the 8 XCDs)."""
    import collections
    import csv
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    for path in paths:
        with open(path) as f:
            for r in csv.DictReader(f):
                name = r["Kernel_Name"]
                if "ddhf::" not in name:
                    continue
                short = name.split("(")[0].replace("void ", "")
                vals[short][r["Counter_Name"]].append(float(r["Counter_Value"]))
    lines = []
    for k in sorted(vals, key=lambda k: -max(sum(v) / len(v) for v in vals[k].values())):
        c = {n: sum(v) / len(v) for n, v in vals[k].items()}
        if not any(t in k for t in ("k_ndft", "k_comb")):
            continue
        lines.append(k)
        for n in sorted(c):
            lines.append(f"  {n:28s} {c[n]:16.6g}")
        w = c.get("SQ_WAVES")
        g = c.get("GRBM_GUI_ACTIVE")
        if w:
            for n, lab in (("SQ_INSTS_VALU", "VALU"), ("SQ_INSTS_SALU", "SALU"),
                           ("SQ_INSTS_LDS", "LDS"), ("SQ_INSTS_MFMA", "MFMA")):
                if n in c:
                    lines.append(f"  -> {lab} instructions per wave  {c[n] / w:12.1f}")
        if g:
            g1 = g / MI355X_XCDS
            if "SQ_ACTIVE_INST_VALU" in c:
                lines.append(f"  -> VALUBusy %                  "
                             f"{100 * c['SQ_ACTIVE_INST_VALU'] / MI355X_CUS / g1:12.1f}")
            if "SQ_VALU_MFMA_BUSY_CYCLES" in c:
                lines.append(f"  -> MfmaUtil %                  "
                             f"{100 * c['SQ_VALU_MFMA_BUSY_CYCLES'] / MI355X_SIMDS / g1:12.1f}")
            if "SQ_LDS_BANK_CONFLICT" in c:
                lines.append(f"  -> LDSBankConflict %           "
                             f"{100 * c['SQ_LDS_BANK_CONFLICT'] / MI355X_CUS / g1:12.1f}")
            lines.append(f"  -> GRBM_GUI_ACTIVE per XCD      {g1:12.6g} cycles")
    print("\n".join(lines), flush=True)


def kernel_source_digest(names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2603_08386_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_tag, digest, profiles_dir=None):
    """HBM bytes per launch from rocprofv3 --pmc (FETCH_SIZE, WRITE_SIZE), scaled by
    a copy-kernel calibration; valid only while the kernel source is unchanged."""
    path = os.path.join(profiles_dir or os.path.join(ROOT, "profiles"),
                        f"traffic_{kernel_tag}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_digest") != digest:
        return None
    return rec.get("bytes_per_launch")


def soft_leg(args, D, synth):
    """Soft comb training step (forward + backward through the library kernels)
    over a batch of labelled 346x260, 50 ms windows; the FP64 oracle's forward +
    backward on a sample of one window's pixels beside it."""
    import torch
    import oracle
    from paper_2603_08386_amd import autograd as AG
    from paper_2603_08386_amd import tune

    wins = [synth.medium_window(400 + i, n_drones=4) for i in range(args.soft_windows)]
    data = [tune.batch(tune.prepare(wins, device="cuda:0"))]  # one graph: one launch each way
    nh = data[0].graph.nh
    ev_h = 0
    for d in data:
        rp, act = d.graph.row_ptr, d.graph.active.long()
        ev_h += int((rp[act + 1] - rp[act]).sum().item()) * nh
    med, sd = tune._score_scale(data, torch.float32)
    beta = 4.0 / sd
    w = torch.full((nh,), 1.0 / nh, device="cuda:0", requires_grad=True)
    tau = torch.tensor([med], device="cuda:0", requires_grad=True)
    stream = torch.cuda.current_stream()
    fwd_ms, bwd_ms, step_ms = [], [], []
    for it in range(2 + args.soft_steps):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(stream)
        loss = tune.bce_loss(data, w, tau, beta)
        e1.record(stream)
        loss.backward()
        e2.record(stream)
        torch.cuda.synchronize()
        w.grad = None
        tau.grad = None
        if it >= 2:
            fwd_ms.append(e0.elapsed_time(e1))
            bwd_ms.append(e1.elapsed_time(e2))
            step_ms.append(e0.elapsed_time(e2))
    ms = float(np.median(step_ms))
    flops = SOFT_FLOP_PER_EVENT_HARMONIC * ev_h
    tflops = flops / (ms * 1e-3) / 1e12
    # oracle: FP64 forward + backward on a uniform sample of one window's pixels
    d0 = data[0]
    G = d0.graph
    rp = G.row_ptr.cpu().numpy()
    t_rel = G.t_rel.cpu().numpy().view(np.uint32)
    sgn = G.sgn.double().cpu().numpy()
    act = G.active.cpu().numpy()
    f0 = G.f0_mhz.cpu().numpy()
    rng = np.random.default_rng(0)
    pick = np.sort(rng.choice(act.size, min(act.size, 160000), replace=False))
    e = np.ones(max(int(rp[-1]), 1))
    dt = np.zeros_like(e)
    wv = np.full(nh, 1.0 / nh)
    t_a = time.perf_counter()
    s, phat, Fr, Fi = oracle.soft_comb_forward(rp, t_rel, sgn, e, dt, act[pick], f0[pick], nh,
                                               G.f_max_mhz, wv, med, beta)
    oracle.soft_comb_backward(rp, t_rel, sgn, e, dt, act[pick], f0[pick], nh, G.f_max_mhz, wv,
                              beta, s, phat, Fr, Fi, np.ones_like(s))
    cpu_s = time.perf_counter() - t_a
    cpu_evh = int(np.sum(rp[act[pick] + 1] - rp[act[pick]])) * nh
    return {
        "workload": f"{args.soft_windows} labelled 346x260 windows, 50 ms, {nh} harmonics",
        "event_harmonics": ev_h, "ms_per_step": ms,
        "fwd_ms": float(np.median(fwd_ms)), "bwd_ms": float(np.median(bwd_ms)),
        "event_harmonics_per_s": ev_h / (ms * 1e-3),
        "roofline": {"bound": "alu", "achieved": tflops, "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": tflops / FP32_PEAK_TFLOPS, "traffic": None,
                     "algorithmic": f"{SOFT_FLOP_PER_EVENT_HARMONIC} FLOP x {ev_h} "
                                    "event-harmonics per training step"},
        "cpu_oracle": {"value": cpu_evh / cpu_s, "unit": "event*harmonics/s", "cores": 1,
                       "kind": "oracle", "sample": f"{pick.size} uniformly sampled pixels of the "
                                                   f"batch, forward + backward, FP64, "
                                                   f"{cpu_s:.1f} s"},
    }


def _oracle_sample(args):
    """One worker of the CPU baseline: oracle NDFT + flatness + comb on its
    share of a fixed random order of active pixels, for about target_s
    seconds.  Returns (pixels done, seconds)."""
    import oracle
    ctx, worker, n_workers, target_s = args
    r, act, grid, params = ctx
    rng = np.random.default_rng(0)
    order = rng.permutation(act.size)[worker::n_workers]
    done, spent, batch = 0, 0.0, 8
    while spent < target_s and done < order.size:
        rows = act[order[done:done + batch]]
        t0 = time.perf_counter()
        P = oracle.ndft_power(r["row_ptr"], r["t_rel"], r["a"], rows, grid)
        oracle.score_rows(P, grid, params)
        spent += time.perf_counter() - t0
        done += rows.size
    return done, spent


_ORACLE_CTX = None


def _oracle_worker(args):
    worker, n_workers, target_s = args
    return _oracle_sample((_ORACLE_CTX, worker, n_workers, target_s))


def cpu_baseline(win, target_s, workers):
    """The FP64 oracle (NDFT + flatness + comb) on a uniform random sample of
    active pixels of the same window, scaled to pixel-bins per second: one
    thread, and `workers` independent processes over disjoint shards of the
    sample (forked before the GPU is touched)."""
    import multiprocessing as mp
    import oracle
    global _ORACLE_CTX
    r = oracle.build_pixel_index(win.x, win.y, win.p, win.t, win.W, win.H, win.t0, win.T_w)
    act = oracle.active_pixels(r["row_ptr"], win.params.n_min)
    K = win.grid.K
    _ORACLE_CTX = (r, act, win.grid, win.params)
    done_pix, spent = _oracle_sample((_ORACLE_CTX, 0, 1, target_s))
    cpu = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    one = dict(value=done_pix * K / spent, unit="pixel*bins/s", cores=1, kind="oracle",
               sample=f"{done_pix} uniformly sampled active pixels of the same window "
                      f"(NDFT power + flatness + comb, FP64, one thread of {os.cpu_count()} "
                      f"on {cpu}), {spent:.1f} s")
    n_w = max(1, min(workers, os.cpu_count() or 1))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(n_w) as pool:
        parts = pool.map(_oracle_worker, [(w, n_w, target_s) for w in range(n_w)])
    wall = time.perf_counter() - t0
    pix = sum(p[0] for p in parts)
    one["all_cores"] = dict(value=pix * K / wall, unit="pixel*bins/s", cores=n_w,
                            kind="oracle", sample=f"{pix} pixels in {n_w} processes over "
                                                  f"disjoint shards of the same sample order, "
                                                  f"{wall:.1f} s wall")
    _ORACLE_CTX = None
    return one


def stream_leg(args, D, synth, launch):
    """p50/p99 frame latency of the streaming step and of a plain recompute."""
    import torch
    from paper_2603_08386_amd.stream import Stream

    W, H, T_w, step_us, pkt_us = 1280, 720, 50_000, 1000, 100
    grid = synth.Grid(f0=10_000, df=1000, K=3991)
    prm = synth.Params(M=4, dk=3, h_min=4, n_min=6, tau_sf=0.89, tau_comb=1.5, a_min=49, alpha=3.0)
    gen = synth.EventStream(seed=5, W=W, H=H, rate_hz=10e6, packet_us=pkt_us)
    per_step = step_us // pkt_us
    warm = max(args.stream_warmup, T_w // step_us + 10)
    n_steps = warm + args.stream_steps
    # one second of stream is generated and replayed shifted by whole seconds
    pool_steps = min(n_steps, 1_000_000 // step_us)
    pool = [gen.next_packet() for _ in range(pool_steps * per_step)]
    cycle_us = pool_steps * step_us

    def packet(i):
        c, j = divmod(i, pool_steps * per_step)
        x, y, p, t = pool[j]
        return x, y, p, t + c * cycle_us

    st = Stream(W, H, T_w, gen.t_origin, grid, prm,
                launch=D.make_launch(launch.kernel, launch.bins_per_lane),
                ring_cap=256, max_step_events=32768, max_touched=32768, max_boxes=256)
    lat, boxes_seen = [], 0
    t_loop0 = None
    n_ev = 0
    for s in range(n_steps):
        if s == warm:
            t_loop0 = time.perf_counter()
        pk = [packet(s * per_step + q) for q in range(per_step)]
        for q in pk[:-1]:
            st.push(*q)
        t_a = time.perf_counter()
        st.push(*pk[-1])
        boxes, nb = st.step(gen.t_origin + (s + 1) * step_us, use_graph=True)
        t_b = time.perf_counter()
        if s >= warm:
            lat.append((t_b - t_a) * 1e3)
            boxes_seen = nb
            n_ev += sum(int(q[3].size) for q in pk)
        if s % 2000 == 0:
            print(f"[bench] stream step {s}/{n_steps}", file=sys.stderr, flush=True)
    t_loop = time.perf_counter() - t_loop0
    stats = st.stats()
    st.close()

    # plain recompute of the same sliding window, at frames spread over the run
    frames = np.linspace(warm, n_steps - 1, max(args.plain_frames, 2)).astype(int)
    wins = []
    for s in frames:
        t_now = gen.t_origin + (s + 1) * step_us
        i0 = max(0, (s + 1) * per_step - T_w // pkt_us)
        pk = [packet(i) for i in range(i0, (s + 1) * per_step)]
        xs = np.concatenate([q[0] for q in pk]); ys = np.concatenate([q[1] for q in pk])
        ps = np.concatenate([q[2] for q in pk]); ts = np.concatenate([q[3] for q in pk])
        keep = (ts >= t_now - T_w) & (ts < t_now)
        wins.append((xs[keep], ys[keep], ps[keep], ts[keep], t_now))
    cap = max(w[0].size for w in wins)
    g = None
    plain = []
    for (xs, ys, ps, ts, t_now) in wins:
        if g is None:
            g = D.Window(xs, ys, ps, ts, W, H, t_now - T_w, T_w, grid, prm, device="cuda:0",
                         launch=launch, capacity=cap)
            g.run()
        torch.cuda.synchronize()
        t_a = time.perf_counter()
        g.reload(xs, ys, ps, ts, t_now - T_w)
        g.run()
        t_b = time.perf_counter()
        plain.append((t_b - t_a) * 1e3)
    return {
        "workload": "stream_1280x720_10Mevps", "window_ms": T_w / 1000, "step_ms": step_us / 1000,
        "packet_us": pkt_us, "steps_timed": args.stream_steps, "steps_warmup": warm,
        "stream_generated_s": pool_steps * step_us / 1e6,
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "mean_ms": float(np.mean(lat)),
        "steps_per_s": args.stream_steps / t_loop, "events_per_s": n_ev / t_loop,
        "active_pixels_last": stats["n_active"], "recomputed_last": stats["n_recomputed"],
        "ring_overflow": stats["ring_overflow"], "touched_overflow": stats["touched_overflow"],
        "boxes_last": boxes_seen,
        "plain_recompute": {"frames": len(plain), "p50_ms": float(np.percentile(plain, 50)),
                            "p99_ms": float(np.percentile(plain, 99)),
                            "events_per_window": cap},
    }


def cadence_leg(args, D, synth):
    """The paper's cadence: the 1280x720, 10 Mev/s stream cut into 33,333 us
    non-overlapping frames (30 FPS), each run through the whole path at integer
    modes k = 0..133 over the frame.  Latency per frame: host clock from the
    push of the packet that completes the frame to its boxes on the host
    (events copied host->device inside it)."""
    from paper_2603_08386_amd import frames as F
    W, H, pkt_us = 1280, 720, 100
    prm = synth.Params(M=4, dk=3, h_min=4, n_min=6, tau_sf=0.89, tau_comb=1.5, a_min=49,
                       alpha=3.0)
    gen = synth.EventStream(seed=5, W=W, H=H, rate_hz=10e6, packet_us=pkt_us)
    per_s = 1_000_000 // pkt_us
    pool = [gen.next_packet() for _ in range(per_s)]    # one second, replayed shifted
    drv = F.FrameDriver(W, H, gen.t_origin, prm, device="cuda:0", capacity=600_000)
    warm = 3
    lat, n_ev, boxes = [], [], []
    i = 0
    while drv.index < warm + args.cadence_frames:
        c, j = divmod(i, per_s)
        x, y, p, t = pool[j]
        t_a = time.perf_counter()
        done = drv.push(x, y, p, t + c * 1_000_000)
        t_b = time.perf_counter()
        for fr in done:
            if fr.index >= warm:
                lat.append((t_b - t_a) * 1e3)
                n_ev.append(fr.n_events)
                boxes.append(fr.n_boxes)
        i += 1
    return {"workload": "frames_1280x720_30fps_modes", "frame_us": F.FRAME_US,
            "modes_K": F.MODES_K, "frames_timed": len(lat),
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(np.mean(lat)), "events_per_frame": float(np.mean(n_ev)),
            "boxes_per_frame": float(np.mean(boxes)),
            "budget_ms": F.FRAME_US / 1000.0}


def main():
    args = parse()
    if args.counter_summary:
        counter_summary(args.counter_summary)
        return
    if args.traffic_summary:
        traffic_summary(args, *args.traffic_summary)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU; multi-GPU runs are not part "
                                   "of it (see DESIGN.md: how the path would shard)"}))
        sys.exit(2)
    from paper_2603_08386_amd import synth

    if args.copy_calibration:
        import torch
        assert torch.cuda.is_available(), "bench.py needs a GPU"
        copy_calibration()
        return
    t_gen = time.time()
    win = getattr(synth, WORKLOADS[args.workload])()
    print(f"[bench] workload {args.workload}: {win.n} events, generated in "
          f"{time.time() - t_gen:.1f}s", file=sys.stderr, flush=True)
    cpu = None
    if args.cpu_seconds > 0:
        # before the GPU is touched: the all-cores leg forks worker processes
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(win, args.cpu_seconds, args.cpu_workers)
    import torch
    from paper_2603_08386_amd import ddhf as D
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    if args.kernel == "auto":
        launch = None
    else:
        kernel = {"valu": D.DDHF_KERNEL_VALU, "mfma": D.DDHF_KERNEL_MFMA,
                  "mfma16": D.DDHF_KERNEL_MFMA16}[args.kernel]
        launch = D.make_launch(kernel, args.bpl, split_events=args.split,
                               persistent=args.persistent, nufft_min_events=args.nufft)
    g = D.window_from_synth(win, device="cuda:0", launch=launch,
                            order_by_cost=bool(args.cost_order))
    stream = torch.cuda.current_stream()
    K = int(win.grid.K)
    tune = None
    if launch is None:
        g.index()
        g.fetch_n_active()
        g.alloc_spectra()
        t0 = time.perf_counter()
        launch, best_ms = g.autotune(cache_path=args.autotune_cache)
        tune = {"launch": [launch.kernel, launch.bins_per_lane, launch.split_events,
                           launch.persistent, launch.nufft_min_events], "best_ms": best_ms,
                "seconds": time.perf_counter() - t0}
        print(f"[bench] autotuned launch {tune}", file=sys.stderr, flush=True)

    scoring = None
    if args.scoring == "auto":
        if g.n_active is None:
            g.index()
            g.fetch_n_active()
        g.launch = launch
        fused, ms_s, ms_f = g.select_scoring()
        scoring = {"fused": fused, "ms_split": ms_s, "ms_fused": ms_f}
        print(f"[bench] scoring {scoring}", file=sys.stderr, flush=True)
    else:
        g.fused = args.scoring == "fused"

    ev = lambda: torch.cuda.Event(enable_timing=True)
    stage_ms = {"index": [], "ndft": [], "comb": [], "detect": []}
    frame_ms = []

    def step(record):
        e0, e1, e1b, e2, e3, e4 = ev(), ev(), ev(), ev(), ev(), ev()
        t_a = time.perf_counter()
        e0.record(stream)
        g.index()
        e1.record(stream)
        na = g.fetch_n_active()
        g.alloc_spectra()
        e1b.record(stream)
        if g.fused:
            g.spectra_and_score()  # one kernel: its time is reported under "ndft"
            e2.record(stream)
        else:
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
    kname = KERNEL_NAMES[int(launch.kernel)]
    tag, kfrag = ndft_tag(kname, launch.bins_per_lane)
    nufft = int(launch.nufft_min_events)
    traffic = (load_traffic(f"{tag}_{args.workload}", kernel_source_digest(TRAFFIC_SOURCES["ndft"]))
               if launch.split_events == 0 and launch.persistent == 0 and nufft == 0 else None)
    # the split-FP16 contraction is priced against the FP16 matrix peak (its own
    # dtype); it executes three FP16 products per FP32 term
    peak = FP16_PEAK_TFLOPS if kname == "mfma16" else FP32_PEAK_TFLOPS
    roof_ndft = {"bound": "alu" if kname == "valu" else "mfma",
                 "kernel": kfrag + (f" + k_nufft (pixels with >= {nufft} events)" if nufft else ""),
                 "achieved": achieved_tflops,
                 "peak": peak, "unit": "TFLOP/s",
                 "frac": achieved_tflops / peak, "traffic": traffic,
                 "ms": ndft_ms, "algorithmic": f"{FLOP_PER_EVENT_BIN} FLOP x {ev_bins} event-bins"}
    comb_ms = float(np.mean(stage_ms["comb"]))
    if g.fused:
        # one kernel forms and scores the spectra; its contraction runs in the
        # split-FP16 form unless the launch names the FP32 matrix kernel, and is
        # priced against that form's own peak (the time includes the comb)
        fkind = "mfma" if kname == "mfma" else "mfma16"
        ftag, _ = fused_tag(fkind)
        fpeak = FP16_PEAK_TFLOPS if fkind == "mfma16" else FP32_PEAK_TFLOPS
        ffrag = (f"k_ndft_comb<{win.params.M}, {win.params.dk}, "
                 f"{'true' if fkind == 'mfma16' else 'false'}>")
        roof_ndft.update({"kernel": f"{ffrag} (spectrum in LDS, flatness and comb)",
                          "bound": "mfma", "peak": fpeak,
                          "frac": achieved_tflops / fpeak,
                          "traffic": load_traffic(f"{ftag}_{args.workload}",
                                                  kernel_source_digest(TRAFFIC_SOURCES["comb"]))})
        roof_comb = None
        dominant = roof_ndft
    else:
        comb_bytes = na * K * 4 + na * 12          # read P once; write sf, snr, bin
        comb_gbs = comb_bytes / (comb_ms * 1e-3) / 1e9
        roof_comb = {"bound": "hbm", "kernel": "k_comb_fast", "achieved": comb_gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": comb_gbs / HBM_PEAK_GBS,
                     "traffic": load_traffic(f"comb_fast_{args.workload}",
                                             kernel_source_digest(TRAFFIC_SOURCES["comb"])),
                     "ms": comb_ms,
                     "algorithmic": f"{comb_bytes} bytes (P read + per-pixel outputs)"}
        dominant = roof_ndft if ndft_ms >= comb_ms else roof_comb

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
                   "ndft_kernel": tag, "bins_per_lane": launch.bins_per_lane,
                   "split_events": launch.split_events, "persistent": launch.persistent,
                   "nufft_min_events": nufft, "cost_order": args.cost_order, "autotune": tune,
                   "scoring": "fused" if g.fused else "split", "scoring_tune": scoring},
        "ndft": {"ms": ndft_ms, "pixel_bins_per_s": na * K / (ndft_ms * 1e-3),
                 "event_bins_per_s": ev_bins / (ndft_ms * 1e-3),
                 "pct_fp32_peak": 100.0 * achieved_tflops / FP32_PEAK_TFLOPS},
        "stages_ms": {k: float(np.mean(v)) for k, v in stage_ms.items()},
        "frame_latency_ms": {"p50": float(np.percentile(frame_ms, 50)),
                             "p99": float(np.percentile(frame_ms, 99)),
                             "path": "whole 100 ms window recomputed per frame, inputs resident"},
        "boxes": nbox,
        "roofline": dominant,
        "rooflines": {"ndft": roof_ndft, "comb": roof_comb},
    }
    if args.stream_steps > 0:
        print("[bench] stream leg", file=sys.stderr, flush=True)
        out["stream"] = stream_leg(args, D, synth, launch)
        out["frame_latency_ms"]["stream_p50"] = out["stream"]["p50_ms"]
        out["frame_latency_ms"]["stream_p99"] = out["stream"]["p99_ms"]
    if args.cadence_frames > 0:
        print("[bench] 30 FPS cadence leg", file=sys.stderr, flush=True)
        out["cadence"] = cadence_leg(args, D, synth)
        out["frame_latency_ms"]["frames_30fps_p50"] = out["cadence"]["p50_ms"]
        out["frame_latency_ms"]["frames_30fps_p99"] = out["cadence"]["p99_ms"]
    if args.soft_windows > 0:
        print("[bench] soft comb leg", file=sys.stderr, flush=True)
        out["soft_comb"] = soft_leg(args, D, synth)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
