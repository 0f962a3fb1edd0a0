"""Pins of the oracle's NDFT power (Eq. 6) against facts outside it:
50-digit brute force, the closed forms of Sec. 3.2 (Eq. 1-5) in event form,
the uniform-sampling special case (a plain DFT), and invariances."""
import math

import mpmath
import numpy as np
import pytest

import oracle
from paper_2603_08386_amd.synth import Grid

mpmath.mp.dps = 50


def csr_one_pixel(t_rel, a):
    t_rel = np.asarray(t_rel, np.uint32)
    a = np.asarray(a, np.float64)
    row_ptr = np.array([0, t_rel.shape[0]], np.int32)
    return row_ptr, t_rel, a, np.array([0], np.int32)


def power_one(t_rel, a, grid):
    rp, t, aa, act = csr_one_pixel(t_rel, a)
    return oracle.ndft_power(rp, t, aa, act, grid)[0]


def rel_err(P, ref, floor):
    return np.max(np.abs(P - ref) / np.maximum(np.abs(ref), floor))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_mpmath_brute_force_hz_grid(seed):
    rng = np.random.default_rng(seed)
    n, K = 17, 29
    t = rng.integers(0, 100_000, size=n)
    a = rng.choice([-1.0, 1.0], size=n) * rng.uniform(0.5, 1.5, size=n)
    grid = Grid(f0=int(rng.integers(0, 5_000_000)), df=int(rng.integers(1, 200_000)), K=K)
    P = power_one(t, a, grid)
    ref = []
    for j in range(K):
        f = mpmath.mpf(grid.f0 + j * grid.df)
        F = mpmath.mpc(0)
        for tt, aa in zip(t, a):
            # unreduced phase: 2 pi f[mHz] t[us] 1e-9
            F += mpmath.mpf(float(aa)) * mpmath.expj(2 * mpmath.pi * f * int(tt) / mpmath.mpf(10) ** 9)
        ref.append(float(abs(F) ** 2))
    ref = np.array(ref)
    assert rel_err(P, ref, np.sum(a * a)) < 1e-12


def test_mpmath_mode_grid_matches_paper_normalisation():
    """Mode grid = Eq. 6 with timestamps mapped to [-pi, pi) over the window
    and integer modes k = 0..K-1 (Sec. 3.5); the power is evaluated in
    mpmath directly in that form."""
    rng = np.random.default_rng(7)
    T_w = 33_333
    n, K = 13, 40
    t = rng.integers(0, T_w, size=n)
    a = rng.choice([-1.0, 1.0], size=n)
    grid = Grid(f0=0, df=1, K=K, mode=1, T_w_us=T_w)
    P = power_one(t, a, grid)
    ref = []
    for k in range(K):
        F = mpmath.mpc(0)
        for tt, aa in zip(t, a):
            tn = 2 * mpmath.pi * mpmath.mpf(int(tt)) / T_w - mpmath.pi
            F += aa * mpmath.expj(k * tn)
        ref.append(float(abs(F) ** 2))
    assert rel_err(P, np.array(ref), n) < 1e-12


def test_coincident_events_give_flat_sum_squared():
    t = np.full(9, 12_345)
    a = np.array([1, 1, -1, 1, 1, 1, -1, 1, 1], float)
    P = power_one(t, a, Grid(f0=1000, df=1000, K=512))
    assert np.allclose(P, a.sum() ** 2, rtol=1e-12, atol=1e-12)


def test_periodic_train_closed_form():
    """C events at phi + m T: P(f) = sin^2(pi f T C) / sin^2(pi f T), so the
    power peaks at C^2 on the fundamental and every harmonic."""
    T, C, phi = 4000, 5, 137  # 250 Hz
    t = phi + T * np.arange(C)
    grid = Grid(f0=1000, df=1000, K=2000)
    P = power_one(t, np.ones(C), grid)
    f_hz = (grid.f0 + grid.df * np.arange(grid.K)) / 1000.0
    x = f_hz * T * 1e-6
    with np.errstate(divide="ignore", invalid="ignore"):
        ref = np.sin(np.pi * x * C) ** 2 / np.sin(np.pi * x) ** 2
    harm = np.isclose(x, np.round(x))
    ref[harm] = C * C
    assert rel_err(P, ref, C) < 1e-9
    for n in range(1, 8):
        assert P[int(250 * n) - 1] == pytest.approx(C * C, rel=1e-12)


@pytest.mark.parametrize("tau", [0.2, 0.25, 0.3])
def test_edge_pairs_reproduce_rotor_line_spectrum(tau):
    """OFF edges at phi + m T and ON edges at phi + (m + tau) T are the
    derivative of the pulse train of Eq. 1, so
      P(f) = 4 sin^2(pi f tau T) sin^2(pi f T C) / sin^2(pi f T)
    and at the harmonics P(n/T) = 4 C^2 sin^2(pi n tau) = C^2 (2 pi n)^2 |c_n|^2
    with |c_n|^2 = (sin(pi n tau) / (pi n))^2 from Eq. 5."""
    T, C, phi = 4000, 6, 55
    tT = int(round(tau * T))
    t = np.concatenate([phi + T * np.arange(C), phi + tT + T * np.arange(C)])
    a = np.concatenate([-np.ones(C), np.ones(C)])
    grid = Grid(f0=1000, df=1000, K=2500)
    P = power_one(t, a, grid)
    f_hz = (grid.f0 + grid.df * np.arange(grid.K)) / 1000.0
    x = f_hz * T * 1e-6
    with np.errstate(divide="ignore", invalid="ignore"):
        comb = np.sin(np.pi * x * C) ** 2 / np.sin(np.pi * x) ** 2
    comb[np.isclose(x, np.round(x))] = C * C
    ref = 4 * np.sin(np.pi * f_hz * tT * 1e-6) ** 2 * comb
    assert rel_err(P, ref, 2 * C) < 1e-9
    for n in range(1, 9):
        cn2 = (math.sin(math.pi * n * tau) / (math.pi * n)) ** 2
        assert P[250 * n - 1] == pytest.approx(C * C * (2 * math.pi * n) ** 2 * cn2, rel=1e-9, abs=1e-9)


def test_uniform_sampling_reduces_to_dft():
    N, dt, ts = 64, 250, 9_001
    rng = np.random.default_rng(3)
    a = rng.normal(size=N)
    t = ts + dt * np.arange(N)
    grid = Grid(f0=0, df=62_500, K=N)  # f_k = k / (N dt)
    P = power_one(t, a, grid)
    ref = np.abs(np.fft.fft(a)) ** 2
    assert rel_err(P, ref, np.sum(a * a)) < 1e-11


def test_invariances():
    rng = np.random.default_rng(11)
    t = rng.integers(0, 50_000, size=40)
    a = rng.choice([-1.0, 1.0], size=40)
    grid = Grid(f0=10_000, df=1000, K=300)
    P = power_one(t, a, grid)
    # polarity flip
    assert np.array_equal(P, power_one(t, -a, grid))
    # shift by one period of every grid phase (1 s for a 1 Hz grid): exact
    assert np.array_equal(P, power_one(t + 1_000_000, a, grid))
    # grid shift by 1 MHz: integer-us timestamps make P 1 MHz periodic
    g2 = Grid(f0=grid.f0 + 1_000_000_000, df=grid.df, K=grid.K)
    assert np.array_equal(P, power_one(t, a, g2))
    # time reversal conjugates F
    tr = 60_000 - t
    assert rel_err(power_one(tr, a, grid), P, 40) < 1e-12
    # arbitrary shift: power unchanged up to rounding
    assert rel_err(power_one(t + 777, a, grid), P, 40) < 1e-11


def test_parseval_mean_power_equals_sum_of_squares():
    """Over a full period of the grid (f = 0 .. 1e6 - 1 Hz for integer-us
    timestamps), the mean of P equals sum a^2 when timestamps are distinct
    modulo 1 s."""
    t = np.array([3, 1000, 250_001, 999_999, 42])
    a = np.array([1.0, -1.0, 0.5, 2.0, -1.5])
    grid = Grid(f0=0, df=1000, K=1_000_000)
    P = power_one(t, a, grid)
    assert P.mean() == pytest.approx(np.sum(a * a), rel=1e-9)


def test_linearity_of_the_transform():
    """F(A u B) = F(A) + F(B): with B a time-shifted copy of A by half a
    period of bin j, the union cancels exactly at that bin."""
    T = 2000  # half period of 250 Hz
    tA = np.array([100, 1234, 5000, 7777])
    t = np.concatenate([tA, tA + T])
    a = np.ones(8)
    grid = Grid(f0=250_000, df=250_000, K=4)  # 250, 500, 750, 1000 Hz
    P = power_one(t, a, grid)
    PA = power_one(tA, np.ones(4), grid)
    assert P[0] == pytest.approx(0.0, abs=1e-20 + 1e-12)   # odd multiple: cancels
    assert P[1] == pytest.approx(4 * PA[1], rel=1e-12)     # even multiple: doubles
    assert P[2] == pytest.approx(0.0, abs=1e-12)
    assert P[3] == pytest.approx(4 * PA[3], rel=1e-12)


def test_overflowing_grid_rejected():
    with pytest.raises(ValueError):
        power_one([1], [1.0], Grid(f0=1 << 40, df=1, K=4))


def test_empty_pixel_gives_zero_power():
    row_ptr = np.array([0, 0], np.int32)
    P = oracle.ndft_power(row_ptr, np.zeros(0, np.uint32), np.zeros(0), np.array([0], np.int32),
                          Grid(f0=1000, df=1000, K=16))
    assert np.all(P == 0)
