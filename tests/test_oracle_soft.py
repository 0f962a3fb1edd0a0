"""Pins of the oracle's soft comb score and its gradients: the forward against
50-digit brute force at non-integer times, and the backward against central
finite differences of the forward."""
import mpmath
import numpy as np
import pytest

import oracle

mpmath.mp.dps = 40


def case(seed=0, n_pix=3, nh=8):
    rng = np.random.default_rng(seed)
    counts = rng.integers(3, 9, size=n_pix)
    row_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    n = int(row_ptr[-1])
    t = rng.integers(0, 50_000, size=n).astype(np.uint32)
    sgn = rng.choice([-1.0, 1.0], size=n)
    e = rng.uniform(0.5, 1.5, size=n)
    dt = rng.normal(0, 3.0, size=n)
    active = np.arange(n_pix, dtype=np.int32)
    f0 = rng.integers(150_000, 400_000, size=n_pix).astype(np.int64)
    w = rng.uniform(0.05, 0.3, size=nh)
    return row_ptr, t, sgn, e, dt, active, f0, nh, 2_000_000, w


def test_forward_matches_mpmath():
    row_ptr, t, sgn, e, dt, active, f0, nh, fmax, w = case(1)
    tau, beta = 0.7, 1.3
    s, ph, fr, fi = oracle.soft_comb_forward(row_ptr, t, sgn, e, dt, active, f0, nh, fmax, w, tau, beta)
    for u in range(len(active)):
        b, en = row_ptr[u], row_ptr[u + 1]
        x = -mpmath.mpf(tau)
        for h in range(1, nh + 1):
            f = h * int(f0[u])
            if f > fmax:
                assert ph[u, h - 1] == 0.0
                continue
            F = mpmath.mpc(0)
            for k in range(b, en):
                th = 2 * mpmath.pi * f * (int(t[k]) + mpmath.mpf(float(dt[k]))) / mpmath.mpf(10) ** 9
                F += mpmath.mpf(float(sgn[k] * e[k])) * mpmath.expj(th)
            P = abs(F) ** 2 / (en - b)
            assert float(P) == pytest.approx(ph[u, h - 1], rel=1e-9, abs=1e-12)
            x += mpmath.mpf(float(w[h - 1])) * P
        assert s[u] == pytest.approx(float(1 / (1 + mpmath.exp(-beta * x))), rel=1e-10)


def test_harmonics_above_fmax_are_masked():
    row_ptr, t, sgn, e, dt, active, f0, nh, fmax, w = case(2)
    f0[:] = 600_000  # harmonics 4.. exceed 2 kHz
    _, ph, _, _ = oracle.soft_comb_forward(row_ptr, t, sgn, e, dt, active, f0, nh, fmax, w, 0.0, 1.0)
    assert np.all(ph[:, 4:] == 0.0) and np.all(ph[:, :3] > 0.0)


@pytest.mark.parametrize("seed", [0, 3])
def test_backward_matches_finite_differences(seed):
    row_ptr, t, sgn, e, dt, active, f0, nh, fmax, w = case(seed)
    tau, beta = 0.9, 0.8
    rng = np.random.default_rng(seed + 10)
    g_s = rng.normal(size=len(active))

    def loss(w_, tau_, e_, dt_):
        s, _, _, _ = oracle.soft_comb_forward(row_ptr, t, sgn, e_, dt_, active, f0, nh, fmax,
                                              w_, tau_, beta)
        return float(np.dot(g_s, s))

    s, ph, fr, fi = oracle.soft_comb_forward(row_ptr, t, sgn, e, dt, active, f0, nh, fmax, w, tau, beta)
    g_w, g_tau, g_e, g_dt = oracle.soft_comb_backward(row_ptr, t, sgn, e, dt, active, f0, nh, fmax,
                                                      w, beta, s, ph, fr, fi, g_s)
    h = 1e-6
    for k in range(nh):
        wp, wm = w.copy(), w.copy(); wp[k] += h; wm[k] -= h
        assert g_w[k] == pytest.approx((loss(wp, tau, e, dt) - loss(wm, tau, e, dt)) / (2 * h), rel=1e-6, abs=1e-9)
    assert g_tau == pytest.approx((loss(w, tau + h, e, dt) - loss(w, tau - h, e, dt)) / (2 * h), rel=1e-6, abs=1e-9)
    for k in range(0, len(e), 3):
        ep, em = e.copy(), e.copy(); ep[k] += h; em[k] -= h
        assert g_e[k] == pytest.approx((loss(w, tau, ep, dt) - loss(w, tau, em, dt)) / (2 * h), rel=1e-5, abs=1e-8)
        hp = 1e-3
        dp, dm = dt.copy(), dt.copy(); dp[k] += hp; dm[k] -= hp
        assert g_dt[k] == pytest.approx((loss(w, tau, e, dp) - loss(w, tau, e, dm)) / (2 * hp), rel=1e-4, abs=1e-9)
