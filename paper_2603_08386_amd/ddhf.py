"""Thin ctypes binding of libddhf.so (include/ddhf.h).

Argument marshalling only: torch tensors provide device memory and the
current HIP stream; every step of the path runs in the library's kernels.
Functions keep the C names.  If the library is missing the import of this
module raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libddhf.so")

DDHF_OK, DDHF_EINVAL, DDHF_ENOSPACE, DDHF_EHIP, DDHF_ETRUNC = 0, 1, 2, 3, 4
DDHF_GRID_HZ, DDHF_GRID_MODES = 0, 1
DDHF_KERNEL_VALU, DDHF_KERNEL_MFMA, DDHF_KERNEL_MFMA16 = 0, 1, 2
DDHF_INDEX_TIME_SORTED = 1
DDHF_DETECT_MAX_CANDIDATES = 1024
DDHF_DETECT_NOALLOC_MAX_PIXELS = 1 << 20


class DdhfError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {status_string(status)} ({status})")
        self.status = status


class Grid(C.Structure):
    _fields_ = [("f0", C.c_int64), ("df", C.c_int64), ("K", C.c_int32), ("mode", C.c_int32),
                ("T_w_us", C.c_int64)]


class Params(C.Structure):
    _fields_ = [("tau_sf", C.c_float), ("tau_comb", C.c_float), ("alpha", C.c_float),
                ("eps_rel", C.c_float), ("M", C.c_int32), ("dk", C.c_int32),
                ("h_min", C.c_int32), ("n_min", C.c_int32), ("a_min", C.c_int32),
                ("reserved", C.c_int32)]


class Box(C.Structure):
    _fields_ = [("x0", C.c_int32), ("y0", C.c_int32), ("x1", C.c_int32), ("y1", C.c_int32),
                ("n_px", C.c_int32), ("f_dom_hz", C.c_float), ("rep_pixel", C.c_int32),
                ("rep_snr", C.c_float)]


class Counters(C.Structure):
    _fields_ = [("n_in", C.c_int64), ("n_kept", C.c_int64), ("out_of_window", C.c_int64),
                ("out_of_sensor", C.c_int64), ("bad_polarity", C.c_int64),
                ("time_unsorted", C.c_int64)]


class Launch(C.Structure):
    _fields_ = [("kernel", C.c_int32), ("bins_per_lane", C.c_int32), ("split_events", C.c_int32),
                ("persistent", C.c_int32), ("grid_waves", C.c_int32),
                ("nufft_min_events", C.c_int32)]


BOX_DTYPE_FIELDS = [f for f, _ in Box._fields_]

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        L.ddhf_status_string.restype = C.c_char_p
        _lib = L
    return _lib


def status_string(s: int) -> str:
    return lib().ddhf_status_string(C.c_int(s)).decode()


def _check(rc: int, where: str):
    if rc != DDHF_OK:
        raise DdhfError(rc, where)


def _p(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def make_grid(g) -> Grid:
    return Grid(int(g.f0), int(g.df), int(g.K), int(g.mode), int(g.T_w_us))


def make_params(p) -> Params:
    return Params(float(p.tau_sf), float(p.tau_comb), float(p.alpha), float(p.eps_rel), int(p.M),
                  int(p.dk), int(p.h_min), int(p.n_min), int(p.a_min), 0)


def make_launch(kernel=DDHF_KERNEL_VALU, bins_per_lane=32, split_events=0, persistent=0,
                grid_waves=0, nufft_min_events=0) -> Launch:
    return Launch(kernel, bins_per_lane, split_events, persistent, grid_waves, nufft_min_events)


def workspace(nbytes: int, device="cuda") -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


# ---------------------------------------------------------------------------
# C entry points (same names; tensors in, status checked)
# ---------------------------------------------------------------------------

def ddhf_build_pixel_index_workspace_size(n, W, H, T_w_us, flags) -> int:
    b = C.c_size_t(0)
    _check(lib().ddhf_build_pixel_index_workspace_size(C.c_int64(n), C.c_int32(W), C.c_int32(H),
                                                       C.c_int64(T_w_us), C.c_int32(flags),
                                                       C.byref(b)), "workspace_size")
    return b.value


def ddhf_build_pixel_index(x, y, p, t_us, w, n, W, H, t0_us, T_w_us, flags, row_ptr, t_rel, a,
                           perm, counters, ws, stream=None):
    rc = lib().ddhf_build_pixel_index(_p(x), _p(y), _p(p), _p(t_us), _p(w), C.c_int64(n),
                                      C.c_int32(W), C.c_int32(H), C.c_int64(t0_us),
                                      C.c_int64(T_w_us), C.c_int32(flags), _p(row_ptr), _p(t_rel),
                                      _p(a), _p(perm), _p(counters), _p(ws),
                                      C.c_size_t(ws.numel()), _stream(stream))
    _check(rc, "ddhf_build_pixel_index")


def ddhf_active_pixels_workspace_size(n_pix) -> int:
    b = C.c_size_t(0)
    _check(lib().ddhf_active_pixels_workspace_size(C.c_int32(n_pix), C.byref(b)), "workspace_size")
    return b.value


def ddhf_active_pixels(row_ptr, n_pix, n_min, order_by_cost, active, n_active, ws, stream=None):
    rc = lib().ddhf_active_pixels(_p(row_ptr), C.c_int32(n_pix), C.c_int32(n_min),
                                  C.c_int32(order_by_cost), _p(active), _p(n_active), _p(ws),
                                  C.c_size_t(ws.numel()), _stream(stream))
    _check(rc, "ddhf_active_pixels")


def ddhf_ndft_workspace_size(n_active, n_events, grid: Grid, launch: Optional[Launch]) -> int:
    b = C.c_size_t(0)
    _check(lib().ddhf_ndft_workspace_size(C.c_int32(n_active), C.c_int64(n_events), C.byref(grid),
                                          C.byref(launch) if launch is not None else None,
                                          C.byref(b)), "workspace_size")
    return b.value


def ddhf_ndft_power(row_ptr, t_rel, a, active, n_active, n_events, grid: Grid, power,
                    launch: Optional[Launch] = None, ws=None, stream=None):
    rc = lib().ddhf_ndft_power(_p(row_ptr), _p(t_rel), _p(a), _p(active), C.c_int32(n_active),
                               C.c_int64(n_events), C.byref(grid), _p(power),
                               C.byref(launch) if launch is not None else None, _p(ws),
                               C.c_size_t(ws.numel() if ws is not None else 0), _stream(stream))
    _check(rc, "ddhf_ndft_power")


def ddhf_autotune_workspace_size(n_active, n_events, grid: Grid) -> int:
    b = C.c_size_t(0)
    _check(lib().ddhf_autotune_workspace_size(C.c_int32(n_active), C.c_int64(n_events),
                                              C.byref(grid), C.byref(b)), "workspace_size")
    return b.value


def ddhf_autotune(row_ptr, t_rel, a, active, n_active, n_events, grid: Grid, power, ws,
                  cache_path: Optional[str] = None, stream=None):
    """Returns (Launch, best_ms); best_ms is -1 on a cache hit."""
    out = Launch()
    ms = C.c_float(0.0)
    rc = lib().ddhf_autotune(_p(row_ptr), _p(t_rel), _p(a), _p(active), C.c_int32(n_active),
                             C.c_int64(n_events), C.byref(grid), _p(power), _p(ws),
                             C.c_size_t(ws.numel()),
                             cache_path.encode() if cache_path else None, C.byref(out),
                             C.byref(ms), _stream(stream))
    _check(rc, "ddhf_autotune")
    return out, ms.value


def ddhf_autotune_scoring(row_ptr, t_rel, a, active, n_active, n_events, grid: Grid,
                          prm: Params, launch: Optional[Launch], power, ws, sf, snr_best,
                          bin_best, stream=None):
    use = C.c_int32(0)
    ms_s, ms_f = C.c_float(0), C.c_float(0)
    rc = lib().ddhf_autotune_scoring(_p(row_ptr), _p(t_rel), _p(a), _p(active),
                                     C.c_int32(n_active), C.c_int64(n_events), C.byref(grid),
                                     C.byref(prm), C.byref(launch) if launch is not None else None,
                                     _p(power), _p(ws), C.c_size_t(ws.numel()), _p(sf),
                                     _p(snr_best), _p(bin_best), C.byref(use), C.byref(ms_s),
                                     C.byref(ms_f), _stream(stream))
    _check(rc, "ddhf_autotune_scoring")
    return bool(use.value), ms_s.value, ms_f.value


def ddhf_comb_score(power, n_active, grid: Grid, prm: Params, sf, snr_best, bin_best,
                    snr_all=None, stream=None):
    rc = lib().ddhf_comb_score(_p(power), C.c_int32(n_active), C.byref(grid), C.byref(prm),
                               _p(sf), _p(snr_best), _p(bin_best), _p(snr_all), _stream(stream))
    _check(rc, "ddhf_comb_score")


def ddhf_ndft_comb(row_ptr, t_rel, a, active, n_active, grid: Grid, prm: Params, sf, snr_best,
                   bin_best, launch: Optional[Launch] = None, stream=None):
    rc = lib().ddhf_ndft_comb(_p(row_ptr), _p(t_rel), _p(a), _p(active), C.c_int32(n_active),
                              C.byref(grid), C.byref(prm),
                              C.byref(launch) if launch is not None else None, _p(sf),
                              _p(snr_best), _p(bin_best), _stream(stream))
    _check(rc, "ddhf_ndft_comb")


def ddhf_detect_workspace_size(W, H) -> int:
    b = C.c_size_t(0)
    _check(lib().ddhf_detect_workspace_size(C.c_int32(W), C.c_int32(H), C.byref(b)),
           "workspace_size")
    return b.value


def ddhf_detect(active, row_ptr, sf, snr_best, bin_best, n_active, W, H, grid: Grid, prm: Params,
                mask, labels, boxes, max_boxes, n_boxes, ws, stream=None):
    rc = lib().ddhf_detect(_p(active), _p(row_ptr), _p(sf), _p(snr_best), _p(bin_best),
                           C.c_int32(n_active), C.c_int32(W), C.c_int32(H), C.byref(grid),
                           C.byref(prm), _p(mask), _p(labels), _p(boxes), C.c_int32(max_boxes),
                           _p(n_boxes), _p(ws), C.c_size_t(ws.numel()), _stream(stream))
    _check(rc, "ddhf_detect")


def ddhf_detect_noalloc(active, row_ptr, sf, snr_best, bin_best, n_active, W, H, grid: Grid,
                        prm: Params, mask, labels, boxes, max_boxes, n_boxes, stream=None):
    rc = lib().ddhf_detect_noalloc(_p(active), _p(row_ptr), _p(sf), _p(snr_best), _p(bin_best),
                                   C.c_int32(n_active), C.c_int32(W), C.c_int32(H),
                                   C.byref(grid), C.byref(prm), _p(mask), _p(labels), _p(boxes),
                                   C.c_int32(max_boxes), _p(n_boxes), _stream(stream))
    _check(rc, "ddhf_detect_noalloc")


# ---------------------------------------------------------------------------
# conveniences: allocate outputs with torch, call the entry points
# ---------------------------------------------------------------------------

def boxes_to_list(boxes_u8: torch.Tensor, n: int):
    """Decode a device box buffer (int32 view, 8 fields per box) on the host."""
    raw = boxes_u8.view(torch.int32)[: 8 * n].cpu().numpy().reshape(n, 8)
    out = []
    import numpy as np
    for r in raw:
        out.append(dict(x0=int(r[0]), y0=int(r[1]), x1=int(r[2]), y1=int(r[3]), n_px=int(r[4]),
                        f_dom_hz=float(np.array([r[5]], np.int32).view(np.float32)[0]),
                        rep_pixel=int(r[6]),
                        rep_snr=float(np.array([r[7]], np.int32).view(np.float32)[0])))
    return out


class Window:
    """Device copy of one event window plus the buffers of the hot path.

    Allocation happens here, once; run() only launches."""

    def __init__(self, x, y, p, t, W, H, t0, T_w, grid, params, w=None, device="cuda",
                 time_sorted=True, launch: Optional[Launch] = None, order_by_cost=False,
                 max_boxes=256, capacity: Optional[int] = None, fused=False):
        import numpy as np

        dev = torch.device(device)
        self.dev = dev
        self.n = int(t.shape[0])
        self.capacity = max(int(capacity) if capacity is not None else self.n, self.n)
        self.W, self.H, self.t0, self.T_w = int(W), int(H), int(t0), int(T_w)
        self.grid = make_grid(grid)
        self.prm = make_params(params)
        self.launch = launch
        # fused: spectrum, flatness and comb in one kernel (ddhf_ndft_comb); no
        # spectra are kept
        self.fused = bool(fused)
        self.order_by_cost = int(order_by_cost)
        self.flags = DDHF_INDEX_TIME_SORTED if time_sorted else 0
        cap = max(self.capacity, 1)
        self.x = torch.empty(cap, dtype=torch.int16, device=dev)
        self.y = torch.empty(cap, dtype=torch.int16, device=dev)
        self.p = torch.empty(cap, dtype=torch.int8, device=dev)
        self.t = torch.empty(cap, dtype=torch.int64, device=dev)
        self.w = None if w is None else torch.empty(cap, dtype=torch.float32, device=dev)
        self._load(x, y, p, t, w)
        npix = self.W * self.H
        self.npix = npix
        self.row_ptr = torch.empty(npix + 1, dtype=torch.int32, device=dev)
        self.t_rel = torch.empty(cap, dtype=torch.int32, device=dev)
        self.a = torch.empty(cap, dtype=torch.float32, device=dev)
        self.perm = torch.empty(cap, dtype=torch.int32, device=dev)
        self.counters = torch.zeros(6, dtype=torch.int64, device=dev)
        self.ws_index = workspace(ddhf_build_pixel_index_workspace_size(
            self.capacity, self.W, self.H, self.T_w, self.flags), dev)
        self.active = torch.empty(max(npix, 1), dtype=torch.int32, device=dev)
        self.n_active_dev = torch.zeros(1, dtype=torch.int32, device=dev)
        self.ws_active = workspace(ddhf_active_pixels_workspace_size(npix), dev)
        self.ws_detect = workspace(ddhf_detect_workspace_size(self.W, self.H), dev)
        self.mask = torch.empty(npix, dtype=torch.uint8, device=dev)
        self.labels = torch.empty(npix, dtype=torch.int32, device=dev)
        self.max_boxes = int(max_boxes)
        self.boxes = torch.empty(max(self.max_boxes, 1) * 32, dtype=torch.uint8, device=dev)
        self.n_boxes = torch.zeros(2, dtype=torch.int32, device=dev)
        self.power = None
        self.sf = None
        self.n_active = None

    def _load(self, x, y, p, t, w=None):
        """Copies host events into the device buffers (u16 coordinates travel as
        int16 with identical bits)."""
        import numpy as np
        n = int(t.shape[0])
        if n > self.capacity:
            raise ValueError(f"{n} events exceed the window capacity {self.capacity}")
        self.n = n
        if n == 0:
            return
        src = [(self.x, np.ascontiguousarray(x, np.uint16).view(np.int16)),
               (self.y, np.ascontiguousarray(y, np.uint16).view(np.int16)),
               (self.p, np.ascontiguousarray(p, np.int8)),
               (self.t, np.ascontiguousarray(t, np.int64))]
        if w is not None:
            src.append((self.w, np.ascontiguousarray(w, np.float32)))
        for dst, arr in src:
            dst[:n].copy_(torch.from_numpy(arr), non_blocking=False)

    def reload(self, x, y, p, t, t0):
        """Replaces the window's events (same sensor, grid and capacity)."""
        self._load(x, y, p, t)
        self.t0 = int(t0)

    # stage 1 + 2
    def index(self, stream=None):
        ddhf_build_pixel_index(self.x, self.y, self.p, self.t, self.w, self.n, self.W, self.H, self.t0,
                               self.T_w, self.flags, self.row_ptr, self.t_rel, self.a, self.perm,
                               self.counters, self.ws_index, stream)
        ddhf_active_pixels(self.row_ptr, self.npix, int(self.prm.n_min), self.order_by_cost,
                           self.active, self.n_active_dev, self.ws_active, stream)

    def fetch_n_active(self) -> int:
        self.n_active = int(self.n_active_dev.item())
        return self.n_active

    def alloc_spectra(self, n_active: Optional[int] = None):
        na = self.n_active if n_active is None else n_active
        K = int(self.grid.K)
        if getattr(self, "sf", None) is None or self.sf.numel() < max(na, 1):
            self.sf = torch.empty(max(na, 1), dtype=torch.float32, device=self.dev)
            self.snr = torch.empty(max(na, 1), dtype=torch.float32, device=self.dev)
            self.bin = torch.empty(max(na, 1), dtype=torch.int32, device=self.dev)
        if self.fused:
            return
        if self.power is None or self.power.numel() < max(na, 1) * K:
            self.power = torch.empty(max(na, 1) * K, dtype=torch.float32, device=self.dev)
            self.ws_ndft = workspace(ddhf_ndft_workspace_size(max(na, 1), self.n, self.grid,
                                                              self.launch), self.dev)

    def autotune(self, cache_path: Optional[str] = None, stream=None):
        """Times the candidate NDFT launches on this window and keeps the best."""
        ws = workspace(ddhf_autotune_workspace_size(self.n_active, self.n, self.grid), self.dev)
        launch, ms = ddhf_autotune(self.row_ptr, self.t_rel, self.a, self.active, self.n_active,
                                   self.n, self.grid, self.power, ws, cache_path, stream)
        self.launch = launch
        self.ws_ndft = workspace(ddhf_ndft_workspace_size(max(self.n_active, 1), self.n,
                                                          self.grid, launch), self.dev)
        return launch, ms

    def select_scoring(self, stream=None):
        """Times the spectra + comb pair (with this window's launch) against the
        fused kernel and keeps the faster; returns (fused, ms_split, ms_fused)."""
        self.fused = False
        self.alloc_spectra()
        use, ms_s, ms_f = ddhf_autotune_scoring(self.row_ptr, self.t_rel, self.a, self.active,
                                                self.n_active, self.n, self.grid, self.prm,
                                                self.launch, self.power, self.ws_ndft, self.sf,
                                                self.snr, self.bin, stream)
        self.fused = bool(use)
        return self.fused, ms_s, ms_f

    def spectra(self, stream=None):
        ddhf_ndft_power(self.row_ptr, self.t_rel, self.a, self.active, self.n_active, self.n,
                        self.grid, self.power, self.launch, self.ws_ndft, stream)

    def score(self, stream=None, snr_all=None):
        ddhf_comb_score(self.power, self.n_active, self.grid, self.prm, self.sf, self.snr,
                        self.bin, snr_all, stream)

    def spectra_and_score(self, stream=None):
        """Flatness and comb scores of every active pixel: the fused kernel, or
        the spectra to HBM and the comb over them."""
        if self.fused:
            # the launch's matrix kernel; split FP16 when it names none
            lk = self.launch
            if lk is not None and lk.kernel not in (DDHF_KERNEL_MFMA, DDHF_KERNEL_MFMA16):
                lk = None
            ddhf_ndft_comb(self.row_ptr, self.t_rel, self.a, self.active, self.n_active,
                           self.grid, self.prm, self.sf, self.snr, self.bin, lk, stream)
        else:
            self.spectra(stream)
            self.score(stream)

    def detect(self, stream=None):
        ddhf_detect(self.active, self.row_ptr, self.sf, self.snr, self.bin, self.n_active, self.W,
                    self.H, self.grid, self.prm, self.mask, self.labels, self.boxes,
                    self.max_boxes, self.n_boxes, self.ws_detect, stream)

    def run(self, stream=None):
        """Whole hot path for this window; returns the host list of boxes."""
        self.index(stream)
        self.fetch_n_active()
        self.alloc_spectra()
        self.spectra_and_score(stream)
        self.detect(stream)
        nb = self.n_boxes.cpu()
        n = min(int(nb[0]), self.max_boxes)
        return boxes_to_list(self.boxes, n), int(nb[0]), int(nb[1])


def window_from_synth(win, **kw) -> Window:
    return Window(win.x, win.y, win.p, win.t, win.W, win.H, win.t0, win.T_w, win.grid,
                  win.params, **kw)
