"""torch.autograd.Function over the soft comb score (ddhf_soft_comb_forward /
ddhf_soft_comb_backward in include/ddhf.h).

The score of active pixel u is
    s_u = sigmoid(beta (sum_h w_h |F_u(h f0_u)|^2 / n_u - tau))
with F_u evaluated at the harmonics of the pixel's dominant frequency f0_u over
its events (sign p_e, weight e_e, time offset dt_e).  Gradients flow to e, dt,
w and tau; they are computed by the library's backward kernel.  float32 and
float64 tensors are supported (float64 serves torch.autograd.gradcheck).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import ddhf as D

_DT = {torch.float32: 0, torch.float64: 1}


@dataclass
class SoftCombGraph:
    """Fixed (non-differentiable) inputs: CSR of the window and per-pixel f0."""
    row_ptr: torch.Tensor   # i32 [W*H + 1]
    t_rel: torch.Tensor     # i32 (u32 bits) [n]
    sgn: torch.Tensor       # float [n], +-1 in CSR order
    active: torch.Tensor    # i32 [n_active]
    f0_mhz: torch.Tensor    # i64 [n_active]
    nh: int = 8
    f_max_mhz: int = 2_000_000
    beta: float = 1.0


def _fwd(G: SoftCombGraph, e, dt, w, tau):
    na = int(G.active.numel())
    dtype = _DT[e.dtype]
    dev = e.device
    s = torch.empty(na, dtype=e.dtype, device=dev)
    phat = torch.empty(na * G.nh, dtype=e.dtype, device=dev)
    F = torch.empty(na * G.nh * 2, dtype=e.dtype, device=dev)
    rc = D.lib().ddhf_soft_comb_forward(
        D._p(G.row_ptr), D._p(G.t_rel), D._p(G.sgn), D._p(e), D._p(dt), D._p(G.active),
        C.c_int32(na), D._p(G.f0_mhz), C.c_int32(G.nh), C.c_int64(G.f_max_mhz), D._p(w),
        D._p(tau), C.c_double(G.beta), C.c_int32(dtype), D._p(s), D._p(phat), D._p(F),
        D._stream())
    D._check(rc, "ddhf_soft_comb_forward")
    return s, phat, F


class SoftComb(torch.autograd.Function):
    @staticmethod
    def forward(ctx, e, dt, w, tau, G: SoftCombGraph):
        e, dt, w, tau = (x.contiguous() for x in (e, dt, w, tau))
        assert e.dtype == dt.dtype == w.dtype == tau.dtype == G.sgn.dtype
        s, phat, F = _fwd(G, e, dt, w, tau)
        ctx.G = G
        ctx.save_for_backward(e, dt, w, tau, s, phat, F)
        return s

    @staticmethod
    def backward(ctx, g_s):
        e, dt, w, tau, s, phat, F = ctx.saved_tensors
        G = ctx.G
        na = int(G.active.numel())
        dtype = _DT[e.dtype]
        dev = e.device
        g_s = g_s.contiguous().to(e.dtype)
        g_w = torch.empty_like(w)
        g_tau = torch.empty_like(tau)
        g_e = torch.zeros_like(e)
        g_dt = torch.zeros_like(dt)
        nbytes = C.c_size_t(0)
        D._check(D.lib().ddhf_soft_comb_backward_workspace_size(C.c_int32(na), C.c_int32(G.nh),
                                                                C.c_int32(dtype), C.byref(nbytes)),
                 "workspace_size")
        ws = D.workspace(nbytes.value, dev)
        rc = D.lib().ddhf_soft_comb_backward(
            D._p(G.row_ptr), D._p(G.t_rel), D._p(G.sgn), D._p(e), D._p(dt), D._p(G.active),
            C.c_int32(na), D._p(G.f0_mhz), C.c_int32(G.nh), C.c_int64(G.f_max_mhz), D._p(w),
            C.c_double(G.beta), C.c_int32(dtype), D._p(s), D._p(phat), D._p(F), D._p(g_s),
            D._p(g_w), D._p(g_tau), D._p(g_e), D._p(g_dt), D._p(ws), C.c_size_t(ws.numel()),
            D._stream())
        D._check(rc, "ddhf_soft_comb_backward")
        return g_e, g_dt, g_w, g_tau, None


def soft_comb(e, dt, w, tau, G: SoftCombGraph):
    return SoftComb.apply(e, dt, w, tau, G)


def graph_from_window(win_dev: "D.Window", nh: int = 8, beta: float = 1.0,
                      dtype=torch.float32) -> SoftCombGraph:
    """Builds the fixed inputs from a device window that has run the hard path
    (index, spectra, comb): f0 of each active pixel is its dominant frequency."""
    na = win_dev.n_active
    n_kept = int(win_dev.row_ptr[-1].item())
    sgn = torch.sign(win_dev.a[:max(n_kept, 1)]).to(dtype)
    bins = win_dev.bin[:na].to(torch.int64)
    f0 = torch.where(bins >= 0, int(win_dev.grid.f0) + bins * int(win_dev.grid.df),
                     torch.zeros_like(bins))
    f_max = int(win_dev.grid.f0) + (int(win_dev.grid.K) - 1) * int(win_dev.grid.df)
    return SoftCombGraph(win_dev.row_ptr, win_dev.t_rel, sgn, win_dev.active[:na].contiguous(),
                         f0.contiguous(), nh, f_max, beta)
