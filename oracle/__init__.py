"""FP64 CPU oracle of the DDHF hot path -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never calls it; the two share no
code.  Every wrapper below forwards to the C functions in ddhf_oracle.c, each of
which cites the part of the paper it writes out.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ddhf_oracle.c")
_LIB = os.path.join(_HERE, "libddhf_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
                               "-o", _LIB, _SRC, "-lm"])
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = C.CDLL(_LIB)
        _lib.orc_build_pixel_index.restype = C.c_int64
        _lib.orc_active_pixels.restype = C.c_int32
        _lib.orc_ndft_power.restype = C.c_int
        _lib.orc_spectral_flatness.restype = C.c_double
        _lib.orc_detect.restype = C.c_int32
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


I64, I32, F64 = C.c_int64, C.c_int32, C.c_double


class Box(C.Structure):
    _fields_ = [("x0", C.c_int32), ("y0", C.c_int32), ("x1", C.c_int32), ("y1", C.c_int32),
                ("n_px", C.c_int32), ("f_dom_hz", C.c_float), ("rep_pixel", C.c_int32),
                ("rep_snr", C.c_float)]


def grid_Q(grid) -> int:
    return 1_000_000_000 if grid.mode == 0 else int(grid.T_w_us)


def build_pixel_index(x, y, p, t, W, H, t0, T_w, w=None):
    """Returns dict(row_ptr, t_rel, a, perm, counters, n_kept)."""
    n = int(t.shape[0])
    x = np.ascontiguousarray(x, np.uint16); y = np.ascontiguousarray(y, np.uint16)
    p = np.ascontiguousarray(p, np.int8); t = np.ascontiguousarray(t, np.int64)
    row_ptr = np.zeros(W * H + 1, np.int32)
    t_rel = np.zeros(max(n, 1), np.uint32)
    a = np.zeros(max(n, 1), np.float64)
    perm = np.zeros(max(n, 1), np.int32)
    cnt = np.zeros(6, np.int64)
    wp = None
    if w is not None:
        w = np.ascontiguousarray(w, np.float32)
        wp = _p(w)
    m = lib().orc_build_pixel_index(I64(n), _p(x), _p(y), _p(p), _p(t), wp, I32(W), I32(H),
                                    I64(t0), I64(T_w), _p(row_ptr), _p(t_rel), _p(a), _p(perm),
                                    _p(cnt))
    if m < 0:
        raise ValueError("bad arguments")
    return dict(row_ptr=row_ptr, t_rel=t_rel[:m], a=a[:m], perm=perm[:m], counters=cnt,
                n_kept=int(m))


def active_pixels(row_ptr, n_min):
    n_pix = row_ptr.shape[0] - 1
    act = np.zeros(max(n_pix, 1), np.int32)
    c = lib().orc_active_pixels(_p(np.ascontiguousarray(row_ptr, np.int32)), I32(n_pix),
                                I32(n_min), _p(act))
    return act[:c].copy()


def ndft_power(row_ptr, t_rel, a, active, grid):
    """FP64 power spectra [n_active, K] (Eq. 6)."""
    active = np.ascontiguousarray(active, np.int32)
    P = np.zeros((active.shape[0], grid.K), np.float64)
    t_rel = np.ascontiguousarray(t_rel, np.uint32)
    a = np.ascontiguousarray(a, np.float64)
    rc = lib().orc_ndft_power(_p(np.ascontiguousarray(row_ptr, np.int32)),
                              _p(t_rel) if t_rel.size else None, _p(a) if a.size else None,
                              _p(active), I32(active.shape[0]), I64(grid.f0), I64(grid.df),
                              I32(grid.K), I64(grid_Q(grid)), _p(P))
    if rc != 0:
        raise ValueError("grid rejected")
    return P


def spectral_flatness(P, eps_rel):
    P = np.ascontiguousarray(P, np.float64)
    return float(lib().orc_spectral_flatness(_p(P), I32(P.shape[0]), F64(eps_rel)))


def comb_score(P, grid, params, want_all=False):
    P = np.ascontiguousarray(P, np.float64)
    K = P.shape[0]
    sb = np.zeros(1, np.float64); bb = np.zeros(1, np.int32)
    allv = np.zeros(K, np.float64) if want_all else None
    lib().orc_comb_score(_p(P), I32(K), I64(grid.f0), I64(grid.df), I32(params.M),
                         I32(params.dk), I32(params.h_min), F64(params.eps_rel), _p(sb), _p(bb),
                         _p(allv) if want_all else None)
    if want_all:
        return float(sb[0]), int(bb[0]), allv
    return float(sb[0]), int(bb[0])


def score_rows(power, grid, params):
    power = np.ascontiguousarray(power, np.float64)
    n, K = power.shape
    sf = np.zeros(n, np.float64); snr = np.zeros(n, np.float64); b = np.zeros(n, np.int32)
    lib().orc_score_rows(_p(power), I32(n), I32(K), I64(grid.f0), I64(grid.df), I32(params.M),
                         I32(params.dk), I32(params.h_min), F64(params.eps_rel), _p(sf),
                         _p(snr), _p(b))
    return sf, snr, b


def detect(active, row_ptr, sf, snr, bin_best, W, H, grid, params, max_boxes=4096):
    """Returns (mask u8 [H*W], labels i32 [H*W], list of box dicts, n_total)."""
    n_active = int(np.asarray(active).shape[0])
    mask = np.zeros(W * H, np.uint8)
    labels = np.zeros(W * H, np.int32)
    out = (Box * max_boxes)()
    n = lib().orc_detect(_p(np.ascontiguousarray(active, np.int32)),
                         _p(np.ascontiguousarray(row_ptr, np.int32)),
                         _p(np.ascontiguousarray(sf, np.float64)),
                         _p(np.ascontiguousarray(snr, np.float64)),
                         _p(np.ascontiguousarray(bin_best, np.int32)), I32(n_active), I32(W),
                         I32(H), I64(grid.f0), I64(grid.df), I32(grid.mode), I64(grid.T_w_us),
                         F64(params.tau_sf), F64(params.tau_comb), F64(params.alpha),
                         I32(params.n_min), I32(params.a_min), _p(mask), _p(labels), out,
                         I32(max_boxes))
    boxes = [dict(x0=b.x0, y0=b.y0, x1=b.x1, y1=b.y1, n_px=b.n_px, f_dom_hz=b.f_dom_hz,
                  rep_pixel=b.rep_pixel, rep_snr=b.rep_snr) for b in out[:min(n, max_boxes)]]
    return mask, labels, boxes, int(n)


def soft_comb_forward(row_ptr, t_rel, sgn, e, dt, active, f0, nh, f_max, w, tau, beta):
    active = np.ascontiguousarray(active, np.int32)
    na = active.shape[0]
    s = np.zeros(na); ph = np.zeros(na * nh); fr = np.zeros(na * nh); fi = np.zeros(na * nh)
    lib().orc_soft_comb_forward(_p(np.ascontiguousarray(row_ptr, np.int32)),
                                _p(np.ascontiguousarray(t_rel, np.uint32)),
                                _p(np.ascontiguousarray(sgn, np.float64)),
                                _p(np.ascontiguousarray(e, np.float64)),
                                _p(np.ascontiguousarray(dt, np.float64)), _p(active), I32(na),
                                _p(np.ascontiguousarray(f0, np.int64)), I32(nh), I64(f_max),
                                _p(np.ascontiguousarray(w, np.float64)), F64(tau), F64(beta),
                                _p(s), _p(ph), _p(fr), _p(fi))
    return s, ph.reshape(na, nh), fr.reshape(na, nh), fi.reshape(na, nh)


def soft_comb_backward(row_ptr, t_rel, sgn, e, dt, active, f0, nh, f_max, w, beta, s, phat,
                       Fre, Fim, g_s):
    active = np.ascontiguousarray(active, np.int32)
    na = active.shape[0]
    n = int(np.asarray(t_rel).shape[0])
    g_w = np.zeros(nh); g_tau = np.zeros(1); g_e = np.zeros(max(n, 1)); g_dt = np.zeros(max(n, 1))
    lib().orc_soft_comb_backward(_p(np.ascontiguousarray(row_ptr, np.int32)),
                                 _p(np.ascontiguousarray(t_rel, np.uint32)),
                                 _p(np.ascontiguousarray(sgn, np.float64)),
                                 _p(np.ascontiguousarray(e, np.float64)),
                                 _p(np.ascontiguousarray(dt, np.float64)), _p(active), I32(na),
                                 _p(np.ascontiguousarray(f0, np.int64)), I32(nh), I64(f_max),
                                 _p(np.ascontiguousarray(w, np.float64)), F64(beta),
                                 _p(np.ascontiguousarray(s, np.float64)),
                                 _p(np.ascontiguousarray(phat, np.float64)),
                                 _p(np.ascontiguousarray(Fre, np.float64)),
                                 _p(np.ascontiguousarray(Fim, np.float64)),
                                 _p(np.ascontiguousarray(g_s, np.float64)), _p(g_w), _p(g_tau),
                                 _p(g_e), _p(g_dt))
    return g_w, float(g_tau[0]), g_e[:n], g_dt[:n]
