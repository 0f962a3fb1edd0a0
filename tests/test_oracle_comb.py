"""Pins of the oracle's spectral flatness (Eq. 7) and median-normalised
harmonic comb (Eq. 8-11) against hand-built spectra with known answers,
scipy's geometric mean, and brute-force enumeration on tiny spectra."""
import numpy as np
import pytest
from scipy.stats import gmean

import oracle
from paper_2603_08386_amd.synth import Grid, Params


def test_flatness_is_one_for_flat_spectrum():
    assert oracle.spectral_flatness(np.full(100, 3.7), 1e-6) == pytest.approx(1.0, rel=1e-14)


def test_flatness_matches_scipy_gmean_and_am_gm():
    rng = np.random.default_rng(0)
    for _ in range(20):
        P = rng.exponential(size=257) * rng.uniform(0.1, 100)
        P[rng.integers(0, 257, size=5)] = 0.0  # zeros hit the floor
        eps = 1e-6
        fl = np.maximum(P, eps * P.mean())
        ref = gmean(fl) / P.mean()
        sf = oracle.spectral_flatness(P, eps)
        assert sf == pytest.approx(ref, rel=1e-12)
        assert 0.0 < sf <= 1.0
        assert oracle.spectral_flatness(P * 1234.5, eps) == pytest.approx(sf, rel=1e-12)


def test_flatness_of_zero_spectrum_is_one():
    assert oracle.spectral_flatness(np.zeros(8), 1e-6) == 1.0


def test_flatness_of_tone_is_small():
    P = np.full(1000, 1e-3)
    P[100] = 1e3
    assert oracle.spectral_flatness(P, 1e-6) < 0.05


def centres(i, grid, M):
    out = []
    for m in range(1, M + 1):
        num = (m - 1) * grid.f0 + m * i * grid.df
        out.append(num // grid.df if num % grid.df == 0 else (2 * num + grid.df) // (2 * grid.df))
    return out


def test_flat_spectrum_scores_one_everywhere():
    grid = Grid(f0=10_000, df=500, K=400)
    prm = Params(M=4, dk=3, h_min=4)
    best, b, allv = oracle.comb_score(np.full(400, 2.5), grid, prm, want_all=True)
    adm = allv > 0
    assert adm.any()
    assert np.allclose(allv[adm], 1.0, rtol=0, atol=1e-15)
    assert best == pytest.approx(1.0) and b == int(np.flatnonzero(adm)[0])


@pytest.mark.parametrize("i0,S", [(30, 9.0), (55, 40.0), (17, 3.0)])
def test_spike_comb_on_unit_floor_scores_its_height(i0, S):
    """Unit floor plus spikes of height S at the M harmonic centres of
    candidate i0: N = S, the complement median is 1, so SNR(i0) = S and it is
    the best candidate."""
    grid = Grid(f0=10_000, df=500, K=600)
    prm = Params(M=4, dk=3, h_min=4)
    P = np.ones(600)
    for c in centres(i0, grid, 4):
        P[c] = S
    best, b, allv = oracle.comb_score(P, grid, prm, want_all=True)
    assert allv[i0] == pytest.approx(S, rel=1e-15)
    assert b == i0 and best == pytest.approx(S)


def test_second_comb_barely_moves_median():
    """Two interleaved rotor combs (Fig. 1(i)): excluding the first comb's
    windows leaves the second comb's few bins in the complement, which does
    not move its median off the floor."""
    grid = Grid(f0=10_000, df=1000, K=1000)
    prm = Params(M=4, dk=3, h_min=4)
    P = np.ones(1000)
    for c in centres(80, grid, 4):
        P[c] = 50.0
    for c in centres(113, grid, 4):
        P[c] = 30.0
    best, b, allv = oracle.comb_score(P, grid, prm, want_all=True)
    assert b == 80 and best == pytest.approx(50.0)
    assert allv[113] == pytest.approx(30.0)


def test_no_admissible_candidate():
    grid = Grid(f0=10_000, df=500, K=20)
    prm = Params(M=4, dk=3, h_min=4)
    best, b = oracle.comb_score(np.ones(20), grid, prm)
    assert b == -1 and best == 0.0


def test_zero_median_uses_floor():
    """A spectrum that is zero off the comb: the baseline falls back to
    eps_rel times the mean power."""
    grid = Grid(f0=0, df=1, K=200, mode=1, T_w_us=1000)
    prm = Params(M=4, dk=1, h_min=4, eps_rel=1e-3)
    P = np.zeros(200)
    for c in centres(20, grid, 4):
        P[c] = 5.0
    best, b = oracle.comb_score(P, grid, prm)
    assert b == 20
    assert best == pytest.approx(5.0 / (1e-3 * P.mean()))


def brute_comb(P, grid, prm):
    K = P.shape[0]
    best, bi, allv = 0.0, -1, np.zeros(K)
    for i in range(K):
        cs = []
        for c in centres(i, grid, prm.M):
            if c - prm.dk < 0 or c + prm.dk > K - 1:
                break
            cs.append(c)
        if i - prm.dk < 0 or len(cs) < prm.h_min or not cs:
            continue
        excl = set()
        N = 0.0
        for c in cs:
            N += max(P[c - prm.dk:c + prm.dk + 1])
            excl.update(range(c - prm.dk, c + prm.dk + 1))
        N /= len(cs)
        comp = sorted((P[k], k) for k in range(K) if k not in excl)
        med = comp[(len(comp) - 1) // 2][0] if comp else 0.0
        den = max(med, prm.eps_rel * P.mean())
        s = N / den if den > 0 else 0.0
        allv[i] = s
        if bi < 0 or s > best:
            best, bi = s, i
    return best, bi, allv


@pytest.mark.parametrize("seed", range(6))
def test_brute_force_tiny_spectra(seed):
    rng = np.random.default_rng(seed)
    K = int(rng.integers(40, 128))
    mode = int(seed % 2)
    grid = Grid(f0=int(rng.integers(0, 3)) * 500 if mode == 0 else 0,
                df=500 if mode == 0 else 1, K=K, mode=mode, T_w_us=10_000)
    prm = Params(M=int(rng.integers(2, 6)), dk=int(rng.integers(0, 3)), h_min=2)
    P = rng.exponential(size=K)
    P[rng.integers(0, K, size=4)] = 0.25  # ties in value
    best, b, allv = oracle.comb_score(P, grid, prm, want_all=True)
    rb, rbi, rall = brute_comb(P, grid, prm)
    assert b == rbi
    assert best == pytest.approx(rb, rel=1e-14)
    assert np.allclose(allv, rall, rtol=1e-14, atol=0)


def test_noninteger_centres_round_half_up():
    grid = Grid(f0=750, df=500, K=200)  # df does not divide f0
    prm = Params(M=3, dk=1, h_min=3)
    rng = np.random.default_rng(1)
    P = rng.exponential(size=200)
    best, b, allv = oracle.comb_score(P, grid, prm, want_all=True)
    rb, rbi, rall = brute_comb(P, grid, prm)
    assert b == rbi and np.allclose(allv, rall, rtol=1e-14, atol=0)
