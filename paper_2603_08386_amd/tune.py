"""Gradient tuning of the soft comb on labelled windows, and a grid-search
reference.

Each labelled window (events plus the generator's rotor-disc mask) first runs
the hard path on the device to get every active pixel's dominant frequency;
the soft comb score s_u = sigmoid(beta (sum_h w_h P^_uh - tau)) is then
trained against the labels with binary cross-entropy, by Adam on (w, tau)
through the library's backward kernel, or scanned over tau at uniform w.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np
import torch

from . import autograd as AG
from . import ddhf as D
from . import synth


@dataclasses.dataclass
class Labelled:
    graph: AG.SoftCombGraph
    label: torch.Tensor      # float [n_active], 1 on rotor pixels
    e: torch.Tensor          # per-event weights (ones)
    dt: torch.Tensor         # per-event time offsets (zeros)


def prepare(windows: List[synth.Window], device="cuda", nh: int = 8, beta: float = 1.0,
            dtype=torch.float32) -> List[Labelled]:
    out = []
    for win in windows:
        g = D.window_from_synth(win, device=device)
        g.run()
        G = AG.graph_from_window(g, nh=nh, beta=beta, dtype=dtype)
        lab = torch.as_tensor(win.label.ravel(), device=device)[G.active.long()].to(dtype)
        n_kept = int(g.row_ptr[-1].item())
        out.append(Labelled(G, lab, torch.ones(max(n_kept, 1), dtype=dtype, device=device),
                            torch.zeros(max(n_kept, 1), dtype=dtype, device=device)))
    return out


def batch(data: List[Labelled]) -> Labelled:
    """Concatenates labelled windows into one graph (pixel and event indices
    offset per window), so a loss over all of them is one forward and one
    backward launch."""
    gs = [d.graph for d in data]
    dev = gs[0].row_ptr.device
    rps, acts = [], []
    ev_off, px_off = 0, 0
    for d in data:
        rp = d.graph.row_ptr.to(torch.int64)
        n_ev = int(rp[-1].item())
        rps.append(rp[:-1] + ev_off)
        acts.append(d.graph.active.to(torch.int64) + px_off)
        ev_off += n_ev
        px_off += rp.numel() - 1
    rps.append(torch.tensor([ev_off], dtype=torch.int64, device=dev))
    assert ev_off < 2**31 and px_off < 2**31
    cut = lambda x, d: x[:int(d.graph.row_ptr[-1].item())]
    G = AG.SoftCombGraph(
        torch.cat(rps).to(torch.int32), torch.cat([cut(d.graph.t_rel, d) for d in data]),
        torch.cat([cut(d.graph.sgn, d) for d in data]), torch.cat(acts).to(torch.int32),
        torch.cat([g.f0_mhz for g in gs]), gs[0].nh, gs[0].f_max_mhz, gs[0].beta)
    return Labelled(G, torch.cat([d.label for d in data]),
                    torch.cat([cut(d.e, d) for d in data]),
                    torch.cat([cut(d.dt, d) for d in data]))


def _score_scale(data: List[Labelled], dtype):
    """Median and spread of the uniform-weight comb sum x = sum_h P^_h / nh over
    all active pixels; they start tau and set beta."""
    xs = []
    nh = data[0].graph.nh
    dev = data[0].e.device
    w = torch.full((nh,), 1.0 / nh, dtype=dtype, device=dev)
    z = torch.zeros(1, dtype=dtype, device=dev)
    for d in data:
        _, phat, _ = AG._fwd(d.graph, d.e, d.dt, w, z)
        xs.append(phat.view(-1, nh) @ w)
    x = torch.cat(xs)
    return float(x.median()), float(x.std().clamp_min(1e-6))


def bce_loss(data: List[Labelled], w, tau, beta) -> torch.Tensor:
    total, count = 0.0, 0
    for d in data:
        G = dataclasses.replace(d.graph, beta=beta)
        s = AG.soft_comb(d.e, d.dt, w, tau, G).clamp(1e-6, 1 - 1e-6)
        total = total + torch.nn.functional.binary_cross_entropy(s, d.label, reduction="sum")
        count += s.numel()
    return total / max(count, 1)


def accuracy(data: List[Labelled], w, tau, beta) -> float:
    hit, count = 0, 0
    with torch.no_grad():
        for d in data:
            G = dataclasses.replace(d.graph, beta=beta)
            s = AG.soft_comb(d.e, d.dt, w, tau, G)
            hit += int(((s > 0.5).to(d.label.dtype) == d.label).sum().item())
            count += s.numel()
    return hit / max(count, 1)


def tune_gradient(data: List[Labelled], steps: int = 60, lr: float = 0.1, dtype=torch.float32,
                  tau0: Optional[float] = None):
    """Adam on scale-free parameters: w = w_raw / nh (w_raw starts at 1) and
    tau = med + sd * theta (theta starts at 0, or at tau0 when given, e.g. a
    grid-search optimum to refine), so one learning rate suits both whatever
    the spectra's scale."""
    med, sd = _score_scale(data, dtype)
    beta = 4.0 / sd
    dev = data[0].e.device
    nh = data[0].graph.nh
    w_raw = torch.ones(nh, dtype=dtype, device=dev, requires_grad=True)
    th0 = 0.0 if tau0 is None else (tau0 - med) / sd
    theta = torch.full((1,), th0, dtype=dtype, device=dev, requires_grad=True)
    opt = torch.optim.Adam([w_raw, theta], lr=lr)
    hist = []
    for _ in range(steps):
        opt.zero_grad()
        loss = bce_loss(data, w_raw / nh, med + sd * theta, beta)
        loss.backward()
        opt.step()
        hist.append(float(loss.item()))
    w = (w_raw / nh).detach()
    tau = (med + sd * theta).detach()
    hist.append(float(bce_loss(data, w, tau, beta).item()))
    return dict(w=w, tau=tau, beta=beta, loss=hist, accuracy=accuracy(data, w, tau, beta))


def tune_grid(data: List[Labelled], n_tau: int = 41, dtype=torch.float32):
    med, sd = _score_scale(data, dtype)
    beta = 4.0 / sd
    dev = data[0].e.device
    nh = data[0].graph.nh
    w = torch.full((nh,), 1.0 / nh, dtype=dtype, device=dev)
    best = None
    with torch.no_grad():
        for t in np.linspace(med - 3 * sd, med + 3 * sd, n_tau):
            tau = torch.tensor([t], dtype=dtype, device=dev)
            loss = float(bce_loss(data, w, tau, beta).item())
            if best is None or loss < best["loss"]:
                best = dict(tau=float(t), loss=loss)
    tau = torch.tensor([best["tau"]], dtype=dtype, device=dev)
    best.update(beta=beta, accuracy=accuracy(data, w, tau, beta))
    return best
