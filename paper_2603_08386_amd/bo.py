"""Bayesian optimisation of the detection hyperparameters (Sec. 4.1,
Table 2): a Gaussian-process surrogate with expected improvement, uniform
priors over the Table 2 search ranges, a random initial design followed by
sequential EI steps, and the detection F1 at IoU 0.5 as the objective.

The objective runs on the device: each labelled window's CSR and NDFT power
(for every pixel with at least the smallest n_min of the range) are computed
once; an evaluation then only rescores the spectra (ddhf_comb_score with the
candidate M, dk, h_min) and redetects (ddhf_detect with the candidate
thresholds, n_min, a_min and alpha).  The surrogate, the acquisition and the
box matching are host code (numpy/scipy)."""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

# Table 2 search space: name, low, high, integer
SPACE: List[Tuple[str, float, float, bool]] = [
    ("tau_sf", 0.3, 0.98, False),
    ("tau_comb", 1.5, 6.0, False),
    ("M", 4, 16, True),
    ("dk", 0, 4, True),
    ("h_min", 2, 8, True),
    ("n_min", 2, 10, True),
    ("a_min", 9, 196, True),
    ("alpha", 3.0, 20.0, False),
]


def decode(u: Sequence[float]) -> Dict[str, float]:
    """Point of the unit cube -> hyperparameter values (integers rounded)."""
    out = {}
    for (name, lo, hi, is_int), x in zip(SPACE, u):
        v = lo + float(np.clip(x, 0.0, 1.0)) * (hi - lo)
        out[name] = int(round(v)) if is_int else v
    return out


def encode(vals: Dict[str, float]) -> np.ndarray:
    return np.array([(vals[n] - lo) / (hi - lo) for (n, lo, hi, _) in SPACE])


# ---------------------------------------------------------------------------
# box matching
# ---------------------------------------------------------------------------

def iou(a, b) -> float:
    """Intersection over union of inclusive boxes (x0, y0, x1, y1)."""
    ix = min(a[2], b[2]) - max(a[0], b[0]) + 1
    iy = min(a[3], b[3]) - max(a[1], b[1]) + 1
    if ix <= 0 or iy <= 0:
        return 0.0
    inter = ix * iy
    area = lambda r: (r[2] - r[0] + 1) * (r[3] - r[1] + 1)
    return inter / float(area(a) + area(b) - inter)


def match(pred, gt, thr: float = 0.5) -> Tuple[int, int, int]:
    """Greedy one-to-one matching by decreasing IoU; a pair counts when its
    IoU is at least thr.  Returns (true positives, false positives, false
    negatives)."""
    pairs = sorted(((iou(p, g), i, j) for i, p in enumerate(pred) for j, g in enumerate(gt)),
                   reverse=True)
    used_p, used_g = set(), set()
    tp = 0
    for v, i, j in pairs:
        if v < thr:
            break
        if i in used_p or j in used_g:
            continue
        used_p.add(i)
        used_g.add(j)
        tp += 1
    return tp, len(pred) - tp, len(gt) - tp


def f1_score(tp: int, fp: int, fn: int) -> float:
    d = 2 * tp + fp + fn
    return 2.0 * tp / d if d else 1.0


# ---------------------------------------------------------------------------
# Gaussian process with a Matern-5/2 ARD kernel, and expected improvement
# ---------------------------------------------------------------------------

def matern52(X1: np.ndarray, X2: np.ndarray, ls: np.ndarray, var: float) -> np.ndarray:
    d = np.sqrt(np.maximum(((X1[:, None, :] - X2[None, :, :]) / ls) ** 2, 0.0).sum(-1))
    r = math.sqrt(5.0) * d
    return var * (1.0 + r + r * r / 3.0) * np.exp(-r)


class GP:
    """Zero-mean GP on standardised targets; hyperparameters (length scales,
    signal variance, noise) by maximum marginal likelihood."""

    def __init__(self, dim: int):
        self.theta = np.concatenate([np.full(dim, math.log(0.3)), [0.0, math.log(1e-2)]])
        self.dim = dim

    def _unpack(self, th):
        return np.exp(th[:self.dim]), math.exp(th[self.dim]), math.exp(th[self.dim + 1])

    def _nll(self, th, X, y):
        ls, var, noise = self._unpack(th)
        Kx = matern52(X, X, ls, var) + (noise + 1e-8) * np.eye(X.shape[0])
        try:
            L = np.linalg.cholesky(Kx)
        except np.linalg.LinAlgError:
            return 1e25
        a = np.linalg.solve(L.T, np.linalg.solve(L, y))
        return 0.5 * y @ a + np.log(np.diag(L)).sum()

    def fit(self, X: np.ndarray, y: np.ndarray, optimise: bool = True):
        from scipy.optimize import minimize
        self.ym, self.ys = float(y.mean()), float(y.std()) or 1.0
        yn = (y - self.ym) / self.ys
        if optimise:
            bounds = [(math.log(0.02), math.log(5.0))] * self.dim + \
                     [(math.log(0.05), math.log(20.0)), (math.log(1e-6), math.log(1.0))]
            best = None
            for start in (self.theta, np.concatenate([np.zeros(self.dim), [0.0, -4.0]])):
                r = minimize(self._nll, start, args=(X, yn), method="L-BFGS-B", bounds=bounds)
                if best is None or r.fun < best.fun:
                    best = r
            self.theta = best.x
        ls, var, noise = self._unpack(self.theta)
        self.X = X
        Kx = matern52(X, X, ls, var) + (noise + 1e-8) * np.eye(X.shape[0])
        self.L = np.linalg.cholesky(Kx)
        self.alpha = np.linalg.solve(self.L.T, np.linalg.solve(self.L, yn))
        return self

    def predict(self, Xs: np.ndarray):
        ls, var, noise = self._unpack(self.theta)
        Ks = matern52(Xs, self.X, ls, var)
        mu = Ks @ self.alpha
        v = np.linalg.solve(self.L, Ks.T)
        s2 = np.maximum(var - (v * v).sum(0), 1e-12)
        return mu * self.ys + self.ym, np.sqrt(s2) * self.ys


def expected_improvement(mu: np.ndarray, sigma: np.ndarray, best: float,
                         xi: float = 0.01) -> np.ndarray:
    """EI of a maximisation: E[max(f - best - xi, 0)] under N(mu, sigma^2)."""
    from scipy.stats import norm
    z = (mu - best - xi) / sigma
    return (mu - best - xi) * norm.cdf(z) + sigma * norm.pdf(z)


@dataclasses.dataclass
class BOResult:
    X: np.ndarray          # unit-cube points evaluated, in order
    y: np.ndarray          # objective values
    best_x: np.ndarray
    best_y: float

    @property
    def best_params(self) -> Dict[str, float]:
        return decode(self.best_x)

    def running_best(self) -> np.ndarray:
        return np.maximum.accumulate(self.y)


def bayes_opt(f: Callable[[np.ndarray], float], dim: int, n_init: int = 50, n_iter: int = 300,
              seed: int = 0, n_cand: int = 4096, refit_every: int = 10,
              x0: Optional[Sequence[np.ndarray]] = None,
              log: Optional[Callable[[int, float], None]] = None) -> BOResult:
    """Maximises f over [0, 1]^dim: n_init uniform random points (plus any x0),
    then n_iter points each maximising EI over random and locally perturbed
    candidates."""
    rng = np.random.default_rng(seed)
    X = [np.asarray(x, float) for x in (x0 or [])]
    X += [rng.random(dim) for _ in range(n_init)]
    y = [f(x) for x in X]
    gp = GP(dim)
    for it in range(n_iter):
        Xa, ya = np.array(X), np.array(y)
        gp.fit(Xa, ya, optimise=(it % refit_every == 0))
        top = Xa[np.argsort(ya)[::-1][:5]]
        cand = np.concatenate([rng.random((n_cand, dim)),
                               np.clip(top[rng.integers(0, top.shape[0], n_cand // 4)] +
                                       rng.normal(0.0, 0.05, (n_cand // 4, dim)), 0.0, 1.0)])
        mu, sd = gp.predict(cand)
        ei = expected_improvement(mu, sd, float(ya.max()))
        xn = cand[int(np.argmax(ei))]
        X.append(xn)
        y.append(f(xn))
        if log is not None and (it + 1) % 25 == 0:
            log(it + 1, max(y))
    Xa, ya = np.array(X), np.array(y)
    k = int(np.argmax(ya))
    return BOResult(Xa, ya, Xa[k], float(ya[k]))


# ---------------------------------------------------------------------------
# the device objective: F1 at IoU 0.5 over labelled windows
# ---------------------------------------------------------------------------

class DetectionObjective:
    """Labelled windows kept on the device with their spectra; f(params)
    rescored and redetected per call.  gt: per window a list of inclusive
    ground-truth boxes (x0, y0, x1, y1)."""

    def __init__(self, windows, gt_boxes, device="cuda:0", min_n: int = 2):
        import torch
        from . import ddhf as D
        self.D = D
        self.torch = torch
        self.wins = []
        self.gt = [list(map(tuple, g)) for g in gt_boxes]
        for win in windows:
            prm = dataclasses.replace(win.params, n_min=min_n)
            g = D.Window(win.x, win.y, win.p, win.t, win.W, win.H, win.t0, win.T_w, win.grid,
                         prm, device=device, launch=D.make_launch(D.DDHF_KERNEL_MFMA, 64),
                         max_boxes=512)
            g.index()
            g.fetch_n_active()
            g.alloc_spectra()
            g.spectra()
            self.wins.append((win, g))
        torch.cuda.synchronize()
        self.evals = 0

    def boxes(self, vals: Dict[str, float]):
        """Per window, the device's boxes for these hyperparameters."""
        D = self.D
        out = []
        for win, g in self.wins:
            prm = dataclasses.replace(win.params, **{k: vals[k] for k in
                                                     ("tau_sf", "tau_comb", "M", "dk", "h_min",
                                                      "n_min", "a_min", "alpha")})
            P = D.make_params(prm)
            D.ddhf_comb_score(g.power, g.n_active, g.grid, P, g.sf, g.snr, g.bin)
            D.ddhf_detect(g.active, g.row_ptr, g.sf, g.snr, g.bin, g.n_active, g.W, g.H, g.grid,
                          P, g.mask, g.labels, g.boxes, g.max_boxes, g.n_boxes, g.ws_detect)
            nb = g.n_boxes.cpu()
            n = min(int(nb[0]), g.max_boxes)
            out.append([(b["x0"], b["y0"], b["x1"], b["y1"]) for b in D.boxes_to_list(g.boxes, n)])
        self.evals += 1
        return out

    def counts(self, vals: Dict[str, float]) -> Tuple[int, int, int]:
        tp = fp = fn = 0
        for pred, gt in zip(self.boxes(vals), self.gt):
            a, b, c = match(pred, gt)
            tp, fp, fn = tp + a, fp + b, fn + c
        return tp, fp, fn

    def f1(self, vals: Dict[str, float]) -> float:
        return f1_score(*self.counts(vals))

    def __call__(self, u: np.ndarray) -> float:
        return self.f1(decode(u))


# ---------------------------------------------------------------------------
# comparison with the gradient-tuned soft comb
# ---------------------------------------------------------------------------

def soft_comb_boxes(windows, w, tau, beta, a_min: int, alpha: float, device="cuda:0"):
    """Boxes from the soft comb score s = sigmoid(beta (sum_h w_h P^_h - tau))
    of every active pixel (f0 from the hard path): the mask is s >= 0.5,
    then the same components, area filter and merge (ddhf_detect with the
    flatness gate open and s in place of the comb SNR)."""
    import dataclasses as dc
    import torch
    from . import autograd as AG
    from . import ddhf as D
    from . import tune
    out = []
    for win in windows:
        d = tune.prepare([win], device=device)[0]
        G = dc.replace(d.graph, beta=beta)
        s = AG.soft_comb(d.e, d.dt, w, tau, G).detach().float().contiguous()
        na = int(s.numel())
        g = D.Window(win.x, win.y, win.p, win.t, win.W, win.H, win.t0, win.T_w, win.grid,
                     win.params, device=device, max_boxes=512)
        g.index()
        g.fetch_n_active()
        assert g.n_active == na
        prm = dc.replace(win.params, tau_sf=1.0, tau_comb=0.5, a_min=int(a_min), alpha=float(alpha))
        sf = torch.zeros(max(na, 1), dtype=torch.float32, device=device)
        b = torch.zeros(max(na, 1), dtype=torch.int32, device=device)
        D.ddhf_detect(g.active, g.row_ptr, sf, s, b, na, g.W, g.H, g.grid, D.make_params(prm),
                      g.mask, g.labels, g.boxes, g.max_boxes, g.n_boxes, g.ws_detect)
        nb = g.n_boxes.cpu()
        n = min(int(nb[0]), g.max_boxes)
        out.append([(q["x0"], q["y0"], q["x1"], q["y1"]) for q in D.boxes_to_list(g.boxes, n)])
    return out


def _f1_of(boxes, gts):
    tp = fp = fn = 0
    for pred, gt in zip(boxes, gts):
        a, b, c = match(pred, gt)
        tp, fp, fn = tp + a, fp + b, fn + c
    return f1_score(tp, fp, fn)


def main():
    """Tunes Table 2 by BO on labelled 346x260 windows and compares, on held-out
    windows, with Table 2's final values, the best random point, and the
    gradient-tuned soft comb.  Prints one JSON line."""
    import argparse
    import json
    import time
    from . import synth, tune

    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=8)
    ap.add_argument("--test", type=int, default=8)
    ap.add_argument("--init", type=int, default=50)
    ap.add_argument("--iter", type=int, default=300)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()
    train = [synth.medium_window(420 + i) for i in range(args.train)]
    test = [synth.medium_window(520 + i) for i in range(args.test)]
    gt = lambda ws: [w.meta["drone_boxes"] for w in ws]
    obj = DetectionObjective(train, gt(train))
    t2 = dict(tau_sf=0.89, tau_comb=1.5, M=4, dk=3, h_min=4, n_min=6, a_min=147, alpha=19.05)
    t0 = time.time()
    import sys
    r = bayes_opt(obj, len(SPACE), n_init=args.init, n_iter=args.iter, seed=args.seed,
                  log=lambda it, b: print(f"[bo] iteration {it}: best F1 {b:.3f}",
                                          file=sys.stderr, flush=True))
    bo_s = time.time() - t0
    rand_best = decode(r.X[int(np.argmax(r.y[:args.init]))])
    held = DetectionObjective(test, gt(test))
    res = {"train_windows": args.train, "test_windows": args.test,
           "evaluations": int(r.y.size), "bo_seconds": bo_s,
           "table2_final": {"params": t2, "f1_train": obj.f1(t2), "f1_test": held.f1(t2)},
           "random_best": {"params": rand_best, "f1_train": float(r.y[:args.init].max()),
                           "f1_test": held.f1(rand_best)},
           "bo_best": {"params": r.best_params, "f1_train": r.best_y,
                       "f1_test": held.f1(r.best_params)}}
    del obj, held
    # gradient-tuned soft comb on the same training windows
    data = tune.prepare(train)
    g = tune.tune_gradient(data, steps=200)
    del data
    for name, am, al in (("table2_area_merge", 147, 19.05),
                         ("bo_area_merge", r.best_params["a_min"], r.best_params["alpha"])):
        res[f"gradient_soft_comb_{name}"] = {
            "a_min": am, "alpha": al,
            "f1_train": _f1_of(soft_comb_boxes(train, g["w"], g["tau"], g["beta"], am, al), gt(train)),
            "f1_test": _f1_of(soft_comb_boxes(test, g["w"], g["tau"], g["beta"], am, al), gt(test))}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
