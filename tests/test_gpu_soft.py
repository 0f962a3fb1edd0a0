"""GPU soft comb (forward + backward through the C ABI and the autograd
Function) against the FP64 oracle, and torch.autograd.gradcheck on the
float64 instantiation of the same kernels."""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_08386_amd import autograd as AG
from paper_2603_08386_amd import ddhf as D
from paper_2603_08386_amd import synth

from gpu_common import DEV, banner

pytestmark = pytest.mark.gpu


def crop_case(seed, W=8, H=8, n=600, dtype=torch.float64):
    """Small synthetic crop: periodic trains plus noise, random f0 per pixel."""
    rng = np.random.default_rng(seed)
    grid = synth.Grid(f0=10_000, df=500, K=3981)
    win = synth.random_window(seed, W, H, 50_000, n, grid, params=synth.Params(n_min=3))
    r = oracle.build_pixel_index(win.x, win.y, win.p, win.t, W, H, win.t0, win.T_w)
    act = oracle.active_pixels(r["row_ptr"], 3)
    f0 = rng.integers(150_000, 400_000, size=act.size).astype(np.int64)
    f0[::5] = 0  # some pixels without a fundamental
    m = r["n_kept"]
    sgn = r["a"].copy()
    e = rng.uniform(0.6, 1.4, size=m)
    dt = rng.normal(0.0, 5.0, size=m)
    w = rng.uniform(0.05, 0.3, size=8)
    tau, beta = 0.8, 0.7
    t = lambda a, dt_: torch.as_tensor(np.ascontiguousarray(a)).to(dt_).to(DEV)
    G = AG.SoftCombGraph(t(r["row_ptr"], torch.int32), t(r["t_rel"].view(np.int32), torch.int32),
                         t(sgn, dtype), t(act, torch.int32), t(f0, torch.int64), 8, 2_000_000,
                         beta)
    host = dict(r=r, act=act, f0=f0, sgn=sgn, e=e, dt=dt, w=w, tau=tau, beta=beta)
    dev = dict(e=t(e, dtype), dt=t(dt, dtype), w=t(w, dtype), tau=t(np.array([tau]), dtype))
    return G, host, dev


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 1e-3)])
def test_soft_comb_matches_oracle(dtype, tol):
    G, h, d = crop_case(1, dtype=dtype)
    banner(f"soft comb vs oracle {dtype}")
    e = d["e"].clone().requires_grad_(True)
    dt = d["dt"].clone().requires_grad_(True)
    w = d["w"].clone().requires_grad_(True)
    tau = d["tau"].clone().requires_grad_(True)
    s = AG.soft_comb(e, dt, w, tau, G)
    g_s = torch.linspace(-1.0, 1.0, s.numel(), dtype=dtype, device=DEV)
    (s * g_s).sum().backward()
    r = h["r"]
    s64, ph, fr, fi = oracle.soft_comb_forward(r["row_ptr"], r["t_rel"], h["sgn"], h["e"], h["dt"],
                                               h["act"], h["f0"], 8, 2_000_000, h["w"], h["tau"],
                                               h["beta"])
    gw, gtau, ge, gdt = oracle.soft_comb_backward(r["row_ptr"], r["t_rel"], h["sgn"], h["e"],
                                                  h["dt"], h["act"], h["f0"], 8, 2_000_000, h["w"],
                                                  h["beta"], s64, ph, fr, fi,
                                                  g_s.double().cpu().numpy())

    def close(got, ref):
        got = got.detach().double().cpu().numpy().ravel()
        ref = np.asarray(ref, np.float64).ravel()
        return np.max(np.abs(got - ref)) <= tol * max(np.max(np.abs(ref)), 1e-30)

    assert close(s, s64)
    assert close(w.grad, gw)
    assert close(tau.grad, [gtau])
    assert close(e.grad, ge)
    assert close(dt.grad, gdt)


def test_soft_comb_gradcheck_fp64():
    G, h, d = crop_case(2, n=250)
    banner("soft comb gradcheck")
    e = d["e"].clone().requires_grad_(True)
    dt = d["dt"].clone().requires_grad_(True)
    w = d["w"].clone().requires_grad_(True)
    tau = d["tau"].clone().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda a, b, c, q: AG.soft_comb(a, b, c, q, G), (e, dt, w, tau))


def test_soft_comb_deterministic():
    G, h, d = crop_case(3, dtype=torch.float32)
    outs = []
    for _ in range(2):
        w = d["w"].clone().requires_grad_(True)
        s = AG.soft_comb(d["e"], d["dt"], w, d["tau"], G)
        s.sum().backward()
        outs.append((s.detach().cpu().numpy(), w.grad.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_soft_comb_on_hard_path_window():
    """f0 from the device hard path on a 346x260 window with 4 drones, a
    clutter band and noise; tau at the median of the uniform-weight comb sum
    and beta = 4 / its spread, so s does not saturate.  The rotor (label)
    pixels score higher than the other active pixels: higher median, and a
    rank AUC of at least 0.95."""
    from paper_2603_08386_amd import tune
    win = synth.medium_window(401)
    banner("soft comb on the hard path's f0")
    data = tune.prepare([win], device=DEV)
    d = data[0]
    G = d.graph
    med, sd = tune._score_scale(data, torch.float32)
    nh = G.nh
    w = torch.full((nh,), 1.0 / nh, device=DEV)
    tau = torch.tensor([med], device=DEV)
    import dataclasses
    s = AG.soft_comb(d.e, d.dt, w, tau, dataclasses.replace(G, beta=4.0 / sd))
    s = s.detach().cpu().numpy()
    lab = d.label.cpu().numpy() > 0.5
    assert np.isfinite(s).all() and (s >= 0).all() and (s <= 1).all()
    assert lab.sum() >= 100 and (~lab).sum() >= 100
    assert 0.05 < np.median(s) < 0.95                  # not saturated
    assert np.median(s[lab]) > np.median(s[~lab]) + 0.2
    # Mann-Whitney AUC: probability a rotor pixel outscores a non-rotor pixel
    ranks = np.empty(s.size)
    ranks[np.argsort(s, kind="stable")] = np.arange(1, s.size + 1)
    n1, n0 = int(lab.sum()), int((~lab).sum())
    auc = (ranks[lab].sum() - n1 * (n1 + 1) / 2) / (n1 * n0)
    banner(f"  rotor {n1}, other {n0}, AUC {auc:.4f}")
    assert auc >= 0.95
    # every rotor pixel has a fundamental inside the blade-pass band
    f0 = G.f0_mhz.cpu().numpy() / 1000.0
    assert np.all((f0[lab] > 100) & (f0[lab] < 900))
